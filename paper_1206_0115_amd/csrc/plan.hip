// Plan construction on the GPU: root box, Morton keys, stable LSD radix sort,
// leaves and cells of every level, near lists and the M2L work tiles.
//
// The octree follows Sec. 3.2 (levels 0..h-1, leaf level h-1) with cells in
// Morton order (Sec. 4.2); near and far lists follow Sec. 2.1.2 (27 near
// cells, at most 189 far cells: children of the parent's near cells that are
// not adjacent).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "device_util.h"
#include "fmm_internal.h"

namespace fmm {

// ------------------------------------------------------------------ scan
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

template <typename T>
__device__ T block_exclusive_scan(T v, T* lds_wave, T* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  T x = v;
  for (int o = 1; o < 64; o <<= 1) {
    T y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) lds_wave[wave] = x;
  __syncthreads();
  T base = 0, all = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) {
    if (w < wave) base += lds_wave[w];
    all += lds_wave[w];
  }
  __syncthreads();
  *total = all;
  return base + x - v;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_tiles_kernel(
    const T* __restrict__ in, T* __restrict__ out, T* __restrict__ sums,
    int64_t n) {
  __shared__ T lds[kScanThreads / 64];
  const int64_t base = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanItems;
  T v[kScanItems];
  T s = 0;
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    v[k] = i < n ? in[i] : T(0);
    s += v[k];
  }
  T total;
  T run = block_exclusive_scan<T>(s, lds, &total);
  for (int k = 0; k < kScanItems; ++k) {
    int64_t i = base + k;
    if (i < n) out[i] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <typename T>
__global__ void scan_add_kernel(T* __restrict__ out, const T* __restrict__ offs,
                                int64_t n) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] += offs[i / kScanTile];
}

// Exclusive scan of n values (in may equal out).  Temporary blocks are kept
// in `tmp` and released by the caller after the stream has drained.
template <typename T>
void exclusive_scan(const T* in, T* out, int64_t n, hipStream_t s,
                    std::vector<void*>& tmp) {
  if (n <= 0) return;
  const int64_t tiles = (n + kScanTile - 1) / kScanTile;
  T* sums = static_cast<T*>(dev_alloc(sizeof(T) * tiles));
  tmp.push_back(sums);
  scan_tiles_kernel<T><<<dim3(unsigned(tiles)), kScanThreads, 0, s>>>(in, out, sums, n);
  FMM_HIP_CHECK(hipGetLastError());
  if (tiles > 1) {
    exclusive_scan<T>(sums, sums, tiles, s, tmp);
    scan_add_kernel<T><<<dim3(unsigned((n + 255) / 256)), 256, 0, s>>>(out, sums, n);
    FMM_HIP_CHECK(hipGetLastError());
  }
}

// ------------------------------------------------------------- bounding box
constexpr int kBoxBlocks = 512;

__global__ __launch_bounds__(256) void bbox_partial_kernel(
    const double* __restrict__ pos, int64_t n, double* __restrict__ part,
    int* __restrict__ bad) {
  __shared__ double smin[3][256], smax[3][256];
  double mn[3] = {INFINITY, INFINITY, INFINITY};
  double mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  int nonfinite = 0;
  for (int64_t i = int64_t(blockIdx.x) * 256 + threadIdx.x; i < n;
       i += int64_t(gridDim.x) * 256) {
    for (int d = 0; d < 3; ++d) {
      double v = pos[3 * i + d];
      if (!isfinite(v)) nonfinite = 1;
      mn[d] = fmin(mn[d], v);
      mx[d] = fmax(mx[d], v);
    }
  }
  if (nonfinite) atomicOr(bad, 1);
  for (int d = 0; d < 3; ++d) {
    smin[d][threadIdx.x] = mn[d];
    smax[d][threadIdx.x] = mx[d];
  }
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o)
      for (int d = 0; d < 3; ++d) {
        smin[d][threadIdx.x] = fmin(smin[d][threadIdx.x], smin[d][threadIdx.x + o]);
        smax[d][threadIdx.x] = fmax(smax[d][threadIdx.x], smax[d][threadIdx.x + o]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int d = 0; d < 3; ++d) {
      part[6 * blockIdx.x + d] = smin[d][0];
      part[6 * blockIdx.x + 3 + d] = smax[d][0];
    }
}

__global__ __launch_bounds__(256) void bbox_final_kernel(const double* __restrict__ part,
                                                         int nb, double* __restrict__ out) {
  __shared__ double s[256];
  for (int d = 0; d < 6; ++d) {
    double v = d < 3 ? INFINITY : -INFINITY;
    for (int b = threadIdx.x; b < nb; b += 256)
      v = d < 3 ? fmin(v, part[6 * b + d]) : fmax(v, part[6 * b + d]);
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
      if (threadIdx.x < o)
        s[threadIdx.x] = d < 3 ? fmin(s[threadIdx.x], s[threadIdx.x + o])
                               : fmax(s[threadIdx.x], s[threadIdx.x + o]);
      __syncthreads();
    }
    if (threadIdx.x == 0) out[d] = s[0];
    __syncthreads();
  }
}

// -------------------------------------------------------------- Morton keys
// k_d = min(floor((x_d - lo_d) / L * 2^(h-1)), 2^(h-1) - 1): IEEE divide, an
// exact scaling by a power of two and floor -- no contraction is possible.
// The root box comes from the device (per-axis min in box[0..2], max in
// box[3..5]); the cube side L = max extent (1 if zero) is formed here in the
// same FP64 operations as on the host.
__device__ __host__ inline double root_side(const double* box) {
  double L = 0.0;
  for (int d = 0; d < 3; ++d) L = fmax(L, box[3 + d] - box[d]);
  return L == 0.0 ? 1.0 : L;
}

__global__ void keys_kernel(const double* __restrict__ pos, int64_t n,
                            const double* __restrict__ box, int bits,
                            uint64_t* __restrict__ keys, int* __restrict__ idx) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double side = double(int64_t(1) << bits);
  const int64_t kmax = (int64_t(1) << bits) - 1;
  const double lo[3] = {box[0], box[1], box[2]};
  const double L = root_side(box);
  uint32_t k3[3];
  for (int d = 0; d < 3; ++d) {
    double u = (pos[3 * i + d] - lo[d]) / L;
    int64_t k = int64_t(floor(u * side));
    k = k > kmax ? kmax : (k < 0 ? 0 : k);
    k3[d] = uint32_t(k);
  }
  keys[i] = morton3(k3[0], k3[1], k3[2], bits);
  idx[i] = int(i);
}

// ------------------------------------------------------- stable radix sort
// LSD radix sort of (key, value) pairs, 8-bit digits.  Stability (equal keys
// keep input order) is what makes the permutation unique: ties are ordered by
// input index.  Per pass: tile histograms, one exclusive scan over the
// digit-major histogram, then a scatter that ranks equal digits in input
// order with wavefront ballots.
constexpr int kRsThreads = 256;
constexpr int kRsItems = 16;
constexpr int kRsTile = kRsThreads * kRsItems;

__global__ __launch_bounds__(kRsThreads) void radix_hist_kernel(
    const uint64_t* __restrict__ keys, int64_t n, int shift, int mask,
    int ntiles, int* __restrict__ hist) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = int64_t(blockIdx.x) * kRsTile;
  for (int it = 0; it < kRsItems; ++it) {
    int64_t i = base + int64_t(it) * kRsThreads + threadIdx.x;
    if (i < n) atomicAdd(&h[int((keys[i] >> shift) & uint64_t(mask))], 1);
  }
  __syncthreads();
  hist[int64_t(threadIdx.x) * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kRsThreads) void radix_scatter_kernel(
    const uint64_t* __restrict__ kin, const int* __restrict__ vin,
    uint64_t* __restrict__ kout, int* __restrict__ vout, int64_t n, int shift,
    int mask, int ntiles, const int* __restrict__ offs) {
  __shared__ int base_d[256];
  __shared__ int wcnt[kRsThreads / 64][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  base_d[tid] = offs[int64_t(tid) * ntiles + blockIdx.x];
  const uint64_t lt = (uint64_t(1) << lane) - 1;
  const int64_t tbase = int64_t(blockIdx.x) * kRsTile;
  for (int it = 0; it < kRsItems; ++it) {
    for (int k = lane; k < 256; k += 64) wcnt[wave][k] = 0;
    const int64_t i = tbase + int64_t(it) * kRsThreads + tid;
    const bool valid = i < n;
    uint64_t key = valid ? kin[i] : 0;
    int val = valid ? vin[i] : 0;
    const int d = valid ? int((key >> shift) & uint64_t(mask)) : 0;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const int rank = __popcll(peers & lt);
    __syncthreads();
    if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    {
      int run = base_d[tid];
      for (int w = 0; w < kRsThreads / 64; ++w) {
        int c = wcnt[w][tid];
        wcnt[w][tid] = run;
        run += c;
      }
      base_d[tid] = run;
    }
    __syncthreads();
    if (valid) {
      const int p = wcnt[wave][d] + rank;
      kout[p] = key;
      vout[p] = val;
    }
    __syncthreads();
  }
}

// Sorts n pairs by the digits of (key >> shift) & mask over `bits` bits.
// Returns the buffers holding the result (either the inputs or the outputs).
static void radix_sort(uint64_t*& k, int*& v, uint64_t*& k2, int*& v2,
                       int64_t n, int bits, hipStream_t s,
                       std::vector<void*>& tmp) {
  if (n <= 1 || bits <= 0) return;
  const int ntiles = ceil_div(n, kRsTile);
  int* hist = static_cast<int*>(dev_alloc(sizeof(int) * 256 * size_t(ntiles)));
  tmp.push_back(hist);
  for (int shift = 0; shift < bits; shift += 8) {
    const int db = std::min(8, bits - shift);
    const int mask = (1 << db) - 1;
    radix_hist_kernel<<<ntiles, kRsThreads, 0, s>>>(k, n, shift, mask, ntiles, hist);
    FMM_HIP_CHECK(hipGetLastError());
    exclusive_scan<int>(hist, hist, int64_t(256) * ntiles, s, tmp);
    radix_scatter_kernel<<<ntiles, kRsThreads, 0, s>>>(k, v, k2, v2, n, shift, mask,
                                                       ntiles, hist);
    FMM_HIP_CHECK(hipGetLastError());
    std::swap(k, k2);
    std::swap(v, v2);
  }
}

// ------------------------------------------------------------- segments
// Unique values of (keys >> shift) over a sorted array: segment flags, their
// exclusive scan, then the unique keys, each segment's first index, and the
// segment of every element.
__global__ void seg_flags_kernel(const uint64_t* __restrict__ keys, int64_t m,
                                 int shift, int* __restrict__ flags) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  flags[i] = (i == 0 || (keys[i] >> shift) != (keys[i - 1] >> shift)) ? 1 : 0;
}

__global__ void seg_emit_kernel(const uint64_t* __restrict__ keys, int64_t m,
                                int shift, const int* __restrict__ flags,
                                const int* __restrict__ pos,
                                uint64_t* __restrict__ ukeys,
                                int* __restrict__ first, int* __restrict__ seg) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int id = pos[i] + flags[i] - 1;
  if (seg) seg[i] = id;
  if (flags[i]) {
    ukeys[id] = keys[i] >> shift;
    first[id] = int(i);
  }
}

__global__ void seg_count_kernel(const int* __restrict__ flags,
                                 const int* __restrict__ pos, int64_t m,
                                 int* __restrict__ count) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *count = pos[m - 1] + flags[m - 1];
}

__global__ void set_int_kernel(int* __restrict__ p, int v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// ------------------------------------------------- all coarser levels at once
// Leaf i of the sorted unique leaf keys k starts a new cell at level l exactly
// when (k[i] >> 3(h-1-l)) != (k[i-1] >> 3(h-1-l)), i.e. at every level from
// h-1-floor(t/3) on, t the highest bit in which k[i] and k[i-1] differ.  One
// pass therefore gives the segment flags of every level l = 0 .. h-2, stored
// level-major: flags[l * nl + i].
// Also counts the cells of every level >= 2 by child parity (the M2L tile
// layout), so that one read-back after the scan brings both.
__global__ __launch_bounds__(256) void level_flags_kernel(const uint64_t* __restrict__ lk,
                                                          int64_t nl, int h,
                                                          int64_t* __restrict__ flags,
                                                          int* __restrict__ pcount) {
  __shared__ int hist[8 * kMaxHeight];
  for (int e = threadIdx.x; e < 8 * kMaxHeight; e += blockDim.x) hist[e] = 0;
  __syncthreads();
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < nl) {
    int first = 0;  // leaf 0 starts a cell at every level
    if (i > 0) first = h - 1 - (63 - __clzll(lk[i] ^ lk[i - 1])) / 3;
    for (int l = 0; l < h - 1; ++l) flags[int64_t(l) * nl + i] = l >= first ? 1 : 0;
    // cells starting at this leaf, levels 2 .. h-1 (every leaf is a cell)
    for (int l = first > 2 ? first : 2; l < h; ++l)
      atomicAdd(&hist[8 * l + int((lk[i] >> (3 * (h - 1 - l))) & 7u)], 1);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 8 * kMaxHeight; e += blockDim.x)
    if (hist[e]) atomicAdd(&pcount[e], hist[e]);
}

struct LevelOut {
  uint64_t* keys[kMaxHeight];
  int* child_start[kMaxHeight];  // [ncell_l + 1] first child at level l+1
  int* parent[kMaxHeight];       // [ncell_l] cell of level l-1 containing it
};

// After an exclusive scan S of the concatenated flags: ncell of every level,
// count[l] = S[(l+1) nl] - S[l nl] (the last level up to the total).
__global__ void level_counts_kernel(const int64_t* __restrict__ flags,
                                    const int64_t* __restrict__ S, int64_t nl, int h,
                                    int64_t* __restrict__ count) {
  const int l = threadIdx.x;
  if (l >= h - 1) return;
  const int64_t end = l + 1 < h - 1 ? S[int64_t(l + 1) * nl]
                                    : S[int64_t(h - 1) * nl - 1] + flags[int64_t(h - 1) * nl - 1];
  count[l] = end - S[int64_t(l) * nl];
}

// Level l (grid y) and leaf i: the unique keys and child offsets of level l
// and the parents of level l+1, all read off the flags and their scan.
__global__ void level_emit_kernel(const uint64_t* __restrict__ lk, int64_t nl, int h,
                                  const int64_t* __restrict__ flags,
                                  const int64_t* __restrict__ S, LevelOut out) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int l = blockIdx.y;
  if (i >= nl) return;
  const int64_t at = int64_t(l) * nl + i;
  const int64_t f = flags[at];
  const int64_t pos = S[at] - S[int64_t(l) * nl];
  const bool leaf1 = l + 1 == h - 1;  // level l+1 is the leaf level
  const bool f1 = leaf1 ? true : flags[at + nl] != 0;
  const int64_t c1 = leaf1 ? i : S[at + nl] - S[int64_t(l + 1) * nl];
  if (f) {
    out.keys[l][pos] = lk[i] >> (3 * (h - 1 - l));
    out.child_start[l][pos] = int(c1);  // a level-l boundary is one at l+1
  }
  if (f1) out.parent[l + 1][c1] = int(pos + f - 1);
}

// child_start[l][ncell_l] = ncell_{l+1} for every level l < h-1
__global__ void level_ends_kernel(LevelOut out, const int64_t* __restrict__ count, int h,
                                  int64_t nl) {
  const int l = threadIdx.x;
  if (l >= h - 1) return;
  out.child_start[l][count[l]] = int(l + 1 < h - 1 ? count[l + 1] : nl);
}

// ------------------------------------------------------------ gathers
__global__ void gather_pos_kernel(const double* __restrict__ pos,
                                  const int* __restrict__ perm, int64_t n,
                                  double* __restrict__ px, double* __restrict__ py,
                                  double* __restrict__ pz) {
  int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t j = perm[i];
  px[i] = pos[3 * j];
  py[i] = pos[3 * j + 1];
  pz[i] = pos[3 * j + 2];
}

// Leaf-local FP32 coordinates for the FP32 near field: x - c_leaf.
__global__ void rel_coords_kernel(const double* __restrict__ px,
                                  const double* __restrict__ py,
                                  const double* __restrict__ pz,
                                  const int* __restrict__ leaf_start,
                                  const uint64_t* __restrict__ leaf_keys,
                                  int64_t nleaf, int bits, double lo0,
                                  double lo1, double lo2, double w,
                                  float4* __restrict__ prel) {
  const int64_t a = blockIdx.x;
  if (a >= nleaf) return;
  int c[3];
  demorton3(leaf_keys[a], bits, c);
  const double cx = lo0 + (c[0] + 0.5) * w, cy = lo1 + (c[1] + 0.5) * w,
               cz = lo2 + (c[2] + 0.5) * w;
  for (int i = leaf_start[a] + threadIdx.x; i < leaf_start[a + 1]; i += blockDim.x)
    prel[i] = make_float4(float(px[i] - cx), float(py[i] - cy), float(pz[i] - cz), 0.f);
}

// ---------------------------------------------------------- lookup tables
struct TableSet {
  const uint64_t* keys[kMaxHeight];
  int* table[kMaxHeight];
  int64_t cum[kMaxHeight + 1];  // prefix sums of the cell counts of the levels
  int nlev;
};

// table[l][key] = index, for the levels of the set (thread = one cell)
__global__ void table_scatter_kernel(TableSet t) {
  const int64_t g = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (g >= t.cum[t.nlev]) return;
  int l = 0;
  while (g >= t.cum[l + 1]) ++l;
  const int64_t i = g - t.cum[l];
  t.table[l][t.keys[l][i]] = int(i);
}

// ------------------------------------------------------------ near lists
// near[a][s], s = (dx+1)*9 + (dy+1)*3 + (dz+1): the leaf at offset (dx,dy,dz)
// or -1.  Also counts directed particle pairs n_a * sum_b n_b.
__global__ void near_kernel(LevelDev leaves, const int* __restrict__ leaf_start,
                            int* __restrict__ near,
                            unsigned long long* __restrict__ pairs) {
  const int a = blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long cnt = 0;
  if (a < leaves.ncell) {
    int c[3];
    demorton3(leaves.keys[a], leaves.bits, c);
    long long src = 0;
    for (int s = 0; s < 27; ++s) {
      const int b = level_find_xyz(leaves, c[0] + s / 9 - 1, c[1] + (s / 3) % 3 - 1,
                                   c[2] + s % 3 - 1);
      near[27 * a + s] = b;
      if (b >= 0) src += leaf_start[b + 1] - leaf_start[b];
    }
    cnt = (unsigned long long)(leaf_start[a + 1] - leaf_start[a]) * (unsigned long long)src;
  }
  for (int o = 32; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o, 64);
  if ((threadIdx.x & 63) == 0 && cnt) atomicAdd(pairs, cnt);
}

// ------------------------------------------------------------ M2L tiles
struct CellLevels {
  const uint64_t* keys[kMaxHeight];
  int64_t off[kMaxHeight + 1];  // global id of each level's first cell
};

// Cells of levels >= 2 (global ids g from off[2]): sort key (level - 2, child
// parity) for the M2L target order, the gid as value.
__global__ __launch_bounds__(256) void parity_keys_kernel(CellLevels c, int h,
                                                          uint64_t* __restrict__ key,
                                                          int* __restrict__ val) {
  const int64_t m = c.off[h] - c.off[2];
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j < m) {
    const int64_t g = c.off[2] + j;
    int l = 2;
    while (g >= c.off[l + 1]) ++l;
    const int par = int(c.keys[l][g - c.off[l]] & 7u);
    key[j] = uint64_t((l - 2) << 3 | par);
    val[j] = int(g);
  }
}

// One workgroup of eight wavefronts per tile.  Lane j of every wavefront owns
// target j; wavefront w looks up the source cells of the slots w, w+8, ...
// (zero row if absent) and marks the slots with at least one source; then
// the marked slots are listed in slot order, each with the mask of its
// 16-target groups that have a source (bit g: targets 16g .. 16g+15), and
// the tile's groups of targets without a source at an active slot are
// counted.
constexpr int kTileThreads = 512;

__global__ __launch_bounds__(kTileThreads) void tile_src_kernel(
    const M2LTile* __restrict__ tiles, const int* __restrict__ tgt,
    const LevelDev* __restrict__ levels, const int64_t* __restrict__ lev_off,
    const signed char* __restrict__ slot_t,  // [8][189][3]
    int zero_row, int* __restrict__ tile_src, unsigned char* __restrict__ act,
    unsigned char* __restrict__ gmask, int* __restrict__ nact, unsigned long long* __restrict__ pairs_level,
    const int* __restrict__ slot_kid, unsigned long long* __restrict__ pairs_kid,
    unsigned long long* __restrict__ active_total,
    unsigned long long* __restrict__ groups) {  // [0] groups at active slots, [1] empty ones
  __shared__ int npair[kSlots];
  __shared__ unsigned char smask[kSlots];
  const int tile = blockIdx.x, j = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const M2LTile T = tiles[tile];
  const LevelDev L = levels[T.level];
  int c[3] = {0, 0, 0};
  const bool have = j < T.count;
  if (have) {
    const int local = tgt[T.first + j] - int(lev_off[T.level]);
    demorton3(L.keys[local], L.bits, c);
  }
  int* out = tile_src + int64_t(tile) * kSlots * kTileN;
  // the lookups of 8 slots are issued before any is used (independent loads
  // in flight instead of one table access at a time)
  constexpr int kStride = kTileThreads / 64, kBatch = 8;
  for (int s0 = wave; s0 < kSlots; s0 += kStride * kBatch) {
    int bs[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int s = s0 + u * kStride;
      bs[u] = -1;
      if (have && s < kSlots) {
        const signed char* t = slot_t + (T.parity * kSlots + s) * 3;
        bs[u] = level_find_xyz(L, c[0] + t[0], c[1] + t[1], c[2] + t[2]);
      }
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int s = s0 + u * kStride;
      if (s >= kSlots) continue;  // the same for the whole wavefront
      out[s * kTileN + j] = bs[u] >= 0 ? bs[u] + int(lev_off[T.level]) : zero_row;
      const uint64_t m = __ballot(bs[u] >= 0);
      if (j == 0) {
        npair[s] = __popcll(m);
        int g = 0;
        for (int q = 0; q < 4; ++q) g |= ((m >> (16 * q)) & 0xffffu) != 0 ? 1 << q : 0;
        smask[s] = (unsigned char)g;
      }
    }
  }
  __syncthreads();
  // active slots in ascending order: wavefront w compacts slots 64w .. 64w+63
  // (a ballot prefix within it, the earlier wavefronts' counts before it)
  __shared__ int wave_active[(kSlots + 63) / 64];
  constexpr int kSlotWaves = (kSlots + 63) / 64;
  static_assert(kSlotWaves * 64 <= kTileThreads, "one thread per slot");
  const int s = threadIdx.x;
  const int k = s < kSlots ? npair[s] : 0;
  const uint64_t m = __ballot(k > 0);
  if (wave < kSlotWaves && j == 0) wave_active[wave] = __popcll(m);
  __syncthreads();
  if (wave < kSlotWaves) {
    int base = 0;
    for (int w = 0; w < wave; ++w) base += wave_active[w];
    if (k > 0) {
      const int pos = base + __popcll(m & ((uint64_t(1) << j) - 1));
      act[int64_t(tile) * kSlots + pos] = (unsigned char)s;
      gmask[int64_t(tile) * kSlots + pos] = smask[s];
      atomicAdd(&pairs_kid[slot_kid[T.parity * kSlots + s]], (unsigned long long)k);
    }
    // pairs of this wavefront's slots, summed across its lanes
    unsigned long long np = (unsigned long long)k;
    for (int o = 32; o > 0; o >>= 1) np += __shfl_xor(np, o, 64);
    if (j == 0 && np) atomicAdd(&pairs_level[T.level], np);
    // groups of targets at the active slots, and those without a source
    const int ngr = (T.count + 15) / 16;
    unsigned long long gt = 0, ge = 0;
    if (k > 0) {
      gt = (unsigned long long)ngr;
      for (int q = 0; q < ngr; ++q) ge += (smask[s] >> q) & 1 ? 0 : 1;
    }
    for (int o = 32; o > 0; o >>= 1) {
      gt += __shfl_xor(gt, o, 64);
      ge += __shfl_xor(ge, o, 64);
    }
    if (j == 0 && gt) {
      atomicAdd(&groups[0], gt);
      if (ge) atomicAdd(&groups[1], ge);
    }
    if (threadIdx.x == 0) {
      int na = 0;
      for (int w = 0; w < kSlotWaves; ++w) na += wave_active[w];
      nact[tile] = na;
      atomicAdd(active_total, (unsigned long long)na);
    }
  }
}

// --------------------------------------------------------------- driver
static inline unsigned grid_for(int64_t n, int b) { return unsigned((n + b - 1) / b); }

void build_plan(fmm_plan_s* p, const double* pos, hipStream_t s) {
  std::vector<void*> tmp;
  struct TmpGuard {
    std::vector<void*>& v;
    hipStream_t s;
    ~TmpGuard() {
      (void)hipStreamSynchronize(s);
      for (void* q : v) dev_free(q);
    }
  } guard{tmp, s};
  auto talloc = [&](size_t b) {
    void* q = dev_alloc(b);
    tmp.push_back(q);
    return q;
  };

  const int64_t n = p->n;
  const int h = p->height;
  const int bits = h - 1;

  // --- root box (the only input-dependent host decision) ---
  const int nb = int(std::min<int64_t>(kBoxBlocks, (n + 255) / 256));
  double* part = static_cast<double*>(talloc(sizeof(double) * 6 * nb + 64));
  double* box = static_cast<double*>(talloc(sizeof(double) * 8));
  int* bad = static_cast<int*>(talloc(sizeof(int)));
  FMM_HIP_CHECK(hipMemsetAsync(bad, 0, sizeof(int), s));
  bbox_partial_kernel<<<nb, 256, 0, s>>>(pos, n, part, bad);
  FMM_HIP_CHECK(hipGetLastError());
  bbox_final_kernel<<<1, 256, 0, s>>>(part, nb, box);
  FMM_HIP_CHECK(hipGetLastError());
  // the box stays on the device until the leaf count comes back: keys are
  // formed from it there (non-finite positions give clamped keys, and the
  // plan is rejected at that first read-back)
  // pinned staging: [0] box (6 doubles), [6] bad flag and leaf count
  char* stage = static_cast<char*>(pinned_staging(4096));
  double* hb = reinterpret_cast<double*>(stage);
  int* hcount = reinterpret_cast<int*>(stage + 64);

  // --- keys and the stable sort ---
  uint64_t* k1 = static_cast<uint64_t*>(talloc(sizeof(uint64_t) * n));
  uint64_t* k2 = static_cast<uint64_t*>(talloc(sizeof(uint64_t) * n));
  int* v1 = static_cast<int*>(talloc(sizeof(int) * n));
  int* v2 = static_cast<int*>(talloc(sizeof(int) * n));
  keys_kernel<<<grid_for(n, 256), 256, 0, s>>>(pos, n, box, bits, k1, v1);
  FMM_HIP_CHECK(hipGetLastError());
  radix_sort(k1, v1, k2, v2, n, 3 * bits, s, tmp);

  p->keys = static_cast<uint64_t*>(p->alloc(sizeof(uint64_t) * n));
  p->perm = static_cast<int*>(p->alloc(sizeof(int) * n));
  FMM_HIP_CHECK(hipMemcpyAsync(p->keys, k1, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
  FMM_HIP_CHECK(hipMemcpyAsync(p->perm, v1, sizeof(int) * n, hipMemcpyDeviceToDevice, s));
  p->px = static_cast<double*>(p->alloc(sizeof(double) * n));
  p->py = static_cast<double*>(p->alloc(sizeof(double) * n));
  p->pz = static_cast<double*>(p->alloc(sizeof(double) * n));
  gather_pos_kernel<<<grid_for(n, 256), 256, 0, s>>>(pos, p->perm, n, p->px, p->py, p->pz);
  FMM_HIP_CHECK(hipGetLastError());

  // --- leaves: the unique keys of the sorted particles ---
  int* flags = static_cast<int*>(talloc(sizeof(int) * n));
  int* scn = static_cast<int*>(talloc(sizeof(int) * n));
  int* cnt_d = static_cast<int*>(talloc(sizeof(int) * 4));
  uint64_t* lk = static_cast<uint64_t*>(talloc(sizeof(uint64_t) * n));
  int* ls = static_cast<int*>(talloc(sizeof(int) * (n + 1)));
  seg_flags_kernel<<<grid_for(n, 256), 256, 0, s>>>(p->keys, n, 0, flags);
  FMM_HIP_CHECK(hipGetLastError());
  exclusive_scan<int>(flags, scn, n, s, tmp);
  seg_emit_kernel<<<grid_for(n, 256), 256, 0, s>>>(p->keys, n, 0, flags, scn, lk, ls, nullptr);
  FMM_HIP_CHECK(hipGetLastError());
  seg_count_kernel<<<1, 64, 0, s>>>(flags, scn, n, cnt_d);
  FMM_HIP_CHECK(hipGetLastError());
  // first read-back: the root box, the non-finite flag and the leaf count
  FMM_HIP_CHECK(hipMemcpyAsync(hb, box, sizeof(double) * 6, hipMemcpyDeviceToHost, s));
  FMM_HIP_CHECK(hipMemcpyAsync(hcount, bad, sizeof(int), hipMemcpyDeviceToHost, s));
  FMM_HIP_CHECK(hipMemcpyAsync(hcount + 1, cnt_d, sizeof(int), hipMemcpyDeviceToHost, s));
  FMM_HIP_CHECK(hipStreamSynchronize(s));
  if (hcount[0]) throw FmmError{FMM_ERR_ARG, "positions contain NaN or Inf"};
  for (int d = 0; d < 3; ++d) p->lo[d] = hb[d];
  const double L = root_side(hb);
  p->L = L;
  p->nleaf = hcount[1];
  const int64_t nl = p->nleaf;
  set_int_kernel<<<1, 64, 0, s>>>(ls + nl, int(n));
  FMM_HIP_CHECK(hipGetLastError());
  p->leaf_start = static_cast<int*>(p->alloc(sizeof(int) * (nl + 1)));
  FMM_HIP_CHECK(hipMemcpyAsync(p->leaf_start, ls, sizeof(int) * (nl + 1),
                               hipMemcpyDeviceToDevice, s));
  LevelView* lev = p->lev;
  lev[h - 1].ncell = nl;
  lev[h - 1].keys = static_cast<uint64_t*>(p->alloc(sizeof(uint64_t) * nl));
  FMM_HIP_CHECK(hipMemcpyAsync(lev[h - 1].keys, lk, sizeof(uint64_t) * nl,
                               hipMemcpyDeviceToDevice, s));
  if (h >= 2) {
    // every coarser level from the leaf keys: flags, one scan, one count
    // read-back, then keys, child offsets and parents in one pass
    const int64_t tot = int64_t(h - 1) * nl;
    int64_t* fl = static_cast<int64_t*>(talloc(sizeof(int64_t) * tot));
    int64_t* S = static_cast<int64_t*>(talloc(sizeof(int64_t) * tot));
    int64_t* cnt = static_cast<int64_t*>(talloc(sizeof(int64_t) * kMaxHeight));
    int* pc = static_cast<int*>(talloc(sizeof(int) * 8 * kMaxHeight));
    FMM_HIP_CHECK(hipMemsetAsync(pc, 0, sizeof(int) * 8 * kMaxHeight, s));
    level_flags_kernel<<<grid_for(nl, 256), 256, 0, s>>>(lk, nl, h, fl, pc);
    FMM_HIP_CHECK(hipGetLastError());
    exclusive_scan<int64_t>(fl, S, tot, s, tmp);
    level_counts_kernel<<<1, 64, 0, s>>>(fl, S, nl, h, cnt);
    FMM_HIP_CHECK(hipGetLastError());
    int64_t* hcnt = reinterpret_cast<int64_t*>(stage + 128);  // pinned
    FMM_HIP_CHECK(hipMemcpyAsync(hcnt, cnt, sizeof(int64_t) * (h - 1), hipMemcpyDeviceToHost, s));
    // per-(level, parity) cell counts for the M2L tiles, in the same read-back
    FMM_HIP_CHECK(hipMemcpyAsync(stage + 512, pc, sizeof(int) * 8 * kMaxHeight,
                                 hipMemcpyDeviceToHost, s));
    FMM_HIP_CHECK(hipStreamSynchronize(s));
    LevelOut out{};
    // every count first: level l's loop iteration sizes level l+1's parents.
    // A tree has one root and at most 8x (and at least as many) cells per
    // level down to the leaves; anything else would make the kernels below
    // write out of bounds.
    for (int l = 0; l < h - 1; ++l) {
      const int64_t below = l + 1 < h - 1 ? hcnt[l + 1] : nl;
      if (hcnt[l] < 1 || hcnt[l] > below || (l == 0 && hcnt[l] != 1))
        throw FmmError{FMM_ERR_HIP, "inconsistent octree level counts"};
      lev[l].ncell = hcnt[l];
    }
    for (int l = 0; l < h - 1; ++l) {
      lev[l].keys = static_cast<uint64_t*>(p->alloc(sizeof(uint64_t) * hcnt[l]));
      lev[l].child_start = static_cast<int*>(p->alloc(sizeof(int) * (hcnt[l] + 1)));
      lev[l + 1].parent = static_cast<int*>(p->alloc(sizeof(int) * lev[l + 1].ncell));
      out.keys[l] = lev[l].keys;
      out.child_start[l] = lev[l].child_start;
      out.parent[l + 1] = lev[l + 1].parent;
    }
    level_emit_kernel<<<dim3(grid_for(nl, 256), unsigned(h - 1)), 256, 0, s>>>(lk, nl, h, fl, S,
                                                                               out);
    FMM_HIP_CHECK(hipGetLastError());
    level_ends_kernel<<<1, 64, 0, s>>>(out, cnt, h, nl);
    FMM_HIP_CHECK(hipGetLastError());
  }
  int64_t off = 0;
  for (int l = 0; l < h; ++l) {
    lev[l].off = off;
    off += lev[l].ncell;
  }
  p->ncell_total = off;
  if (off >= (int64_t(1) << 31) - 1) throw FmmError{FMM_ERR_ARG, "too many cells"};

  // dense lookup tables for levels with at most 2^24 key slots, one block
  LevelDev ldev[kMaxHeight];
  TableSet ts{};
  int64_t tslots = 0;
  for (int l = 0; l < h; ++l) {
    ldev[l] = {lev[l].keys, nullptr, int(lev[l].ncell), l};
    if (3 * l <= 24) tslots += int64_t(1) << (3 * l);
  }
  int* tables = static_cast<int*>(p->alloc(sizeof(int) * tslots));
  FMM_HIP_CHECK(hipMemsetAsync(tables, 0xff, sizeof(int) * tslots, s));  // all -1
  tslots = 0;
  for (int l = 0; l < h && 3 * l <= 24; ++l) {
    lev[l].lookup = tables + tslots;
    ldev[l].table = lev[l].lookup;
    ts.keys[ts.nlev] = lev[l].keys;
    ts.table[ts.nlev] = lev[l].lookup;
    ts.cum[ts.nlev + 1] = ts.cum[ts.nlev] + lev[l].ncell;
    ++ts.nlev;
    tslots += int64_t(1) << (3 * l);
  }
  if (ts.cum[ts.nlev] > 0) {
    table_scatter_kernel<<<grid_for(ts.cum[ts.nlev], 256), 256, 0, s>>>(ts);
    FMM_HIP_CHECK(hipGetLastError());
  }

  // --- near lists ---
  // counters: far pairs per level, near pairs, active M2L slots, then far
  // pairs per operator
  const size_t ncount = kMaxHeight + 2 + kOffsets + 2;
  unsigned long long* counters =
      static_cast<unsigned long long*>(talloc(sizeof(unsigned long long) * ncount));
  FMM_HIP_CHECK(hipMemsetAsync(counters, 0, sizeof(unsigned long long) * ncount, s));
  p->near = static_cast<int*>(p->alloc(sizeof(int) * 27 * nl));
  near_kernel<<<grid_for(nl, 256), 256, 0, s>>>(ldev[h - 1], p->leaf_start, p->near,
                                                counters + kMaxHeight);
  FMM_HIP_CHECK(hipGetLastError());

  // --- leaf-local FP32 coordinates ---
  p->prel = static_cast<float4*>(p->alloc(sizeof(float4) * n));
  rel_coords_kernel<<<unsigned(nl), 64, 0, s>>>(p->px, p->py, p->pz, p->leaf_start,
                                               lev[h - 1].keys, nl, bits, p->lo[0],
                                               p->lo[1], p->lo[2],
                                               L / double(int64_t(1) << bits), p->prel);
  FMM_HIP_CHECK(hipGetLastError());

  // --- M2L tiles: targets of each level >= 2 grouped by child parity ---
  if (h >= 3) {
    const int64_t ntgt = p->ncell_total - lev[2].off;
    p->tgt = static_cast<int*>(p->alloc(sizeof(int) * ntgt));
    // one stable radix pass by (level - 2, parity): within a group the
    // cells stay in Morton order
    CellLevels cl{};
    for (int l = 0; l < h; ++l) {
      cl.keys[l] = lev[l].keys;
      cl.off[l] = lev[l].off;
    }
    cl.off[h] = p->ncell_total;
    uint64_t* pk1 = static_cast<uint64_t*>(talloc(sizeof(uint64_t) * ntgt));
    uint64_t* pk2 = static_cast<uint64_t*>(talloc(sizeof(uint64_t) * ntgt));
    int* pv1 = static_cast<int*>(talloc(sizeof(int) * ntgt));
    int* pv2 = static_cast<int*>(talloc(sizeof(int) * ntgt));
    parity_keys_kernel<<<grid_for(ntgt, 256), 256, 0, s>>>(cl, h, pk1, pv1);
    FMM_HIP_CHECK(hipGetLastError());
    int kbits = 3;
    while ((1 << (kbits - 3)) < h - 2) ++kbits;
    radix_sort(pk1, pv1, pk2, pv2, ntgt, kbits, s, tmp);
    FMM_HIP_CHECK(hipMemcpyAsync(p->tgt, pv1, sizeof(int) * ntgt, hipMemcpyDeviceToDevice, s));
    // counts read back with the level counts (level_flags_kernel)
    const int* hpc = reinterpret_cast<const int*>(stage + 512);
    // finest level first: the largest tiles' work is scheduled before the
    // coarse levels fill in the tail.  Within a level the parities take
    // turns: the k-th tile of every parity covers about the same region of
    // space, so the eight run side by side (on one XCD, whose L2 then serves
    // the source multipoles they share) instead of one parity sweeping the
    // whole level after another.
    std::vector<M2LTile> tiles;
    for (int l = h - 1; l >= 2; --l) {
      int64_t start[8];
      int kmax = 0;
      start[0] = lev[l].off - lev[2].off;
      for (int par = 0; par < 8; ++par) {
        if (par > 0) start[par] = start[par - 1] + hpc[8 * l + par - 1];
        kmax = std::max(kmax, hpc[8 * l + par]);
      }
      for (int k = 0; k < kmax; k += kTileN)
        for (int par = 0; par < 8; ++par) {
          const int c = hpc[8 * l + par];
          if (k < c) tiles.push_back({l, par, int(start[par] + k), std::min(kTileN, c - k)});
        }
    }
    p->ntiles = int64_t(tiles.size());
    p->tiles_host = tiles;
    if (p->ntiles > 0) {
      // every earlier transfer through the staging buffer has completed (the
      // level-count read-back waited for them), so it may grow here; layout
      // from 4 KiB on:
      // level tables, level offsets, then the tiles
      const size_t tbytes = sizeof(M2LTile) * tiles.size();
      stage = static_cast<char*>(pinned_staging(4096 + 2048 + tbytes));
      LevelDev* hld = reinterpret_cast<LevelDev*>(stage + 4096);
      int64_t* hoff = reinterpret_cast<int64_t*>(stage + 4096 + 1024);
      M2LTile* htiles = reinterpret_cast<M2LTile*>(stage + 4096 + 2048);
      static_assert(sizeof(LevelDev) * kMaxHeight <= 1024 && sizeof(int64_t) * kMaxHeight <= 1024,
                    "staging layout");
      std::memcpy(htiles, tiles.data(), tbytes);
      p->tiles = static_cast<M2LTile*>(p->alloc(tbytes));
      FMM_HIP_CHECK(hipMemcpyAsync(p->tiles, htiles, tbytes, hipMemcpyHostToDevice, s));
      p->tile_src = static_cast<int*>(p->alloc(sizeof(int) * size_t(p->ntiles) * kSlots * kTileN));
      p->tile_act = static_cast<unsigned char*>(p->alloc(size_t(p->ntiles) * kSlots));
      p->tile_gmask = static_cast<unsigned char*>(p->alloc(size_t(p->ntiles) * kSlots));
      p->tile_nact = static_cast<int*>(p->alloc(sizeof(int) * p->ntiles));
      LevelDev* ld_d = static_cast<LevelDev*>(talloc(sizeof(LevelDev) * kMaxHeight));
      int64_t* off_d = static_cast<int64_t*>(talloc(sizeof(int64_t) * kMaxHeight));
      for (int l = 0; l < kMaxHeight; ++l) {
        hoff[l] = l < h ? lev[l].off : 0;
        hld[l] = ldev[l];
      }
      FMM_HIP_CHECK(hipMemcpyAsync(ld_d, hld, sizeof(LevelDev) * kMaxHeight,
                                   hipMemcpyHostToDevice, s));
      FMM_HIP_CHECK(hipMemcpyAsync(off_d, hoff, sizeof(int64_t) * kMaxHeight,
                                   hipMemcpyHostToDevice, s));
      tile_src_kernel<<<unsigned(p->ntiles), kTileThreads, 0, s>>>(
          p->tiles, p->tgt, ld_d, off_d, p->ops->slot_t,
          int(p->ncell_total), p->tile_src, p->tile_act, p->tile_gmask, p->tile_nact, counters,
          p->ops->slot_kid, counters + kMaxHeight + 2, counters + kMaxHeight + 1,
          counters + kMaxHeight + 2 + kOffsets);
      FMM_HIP_CHECK(hipGetLastError());
    }
  }

  // --- statistics ---
  // statistics in the staging buffer's first 4 KiB (the box and counts
  // there are no longer needed)
  static_assert(sizeof(unsigned long long) * (kMaxHeight + 4 + kOffsets) <= 4096, "staging");
  unsigned long long* hc = reinterpret_cast<unsigned long long*>(stage);
  FMM_HIP_CHECK(hipMemcpyAsync(hc, counters, sizeof(unsigned long long) * (kMaxHeight + 4 + kOffsets),
                               hipMemcpyDeviceToHost, s));
  // read by plan_stats after the caller's next synchronisation of s (no
  // wait here: nothing the plan builds next needs them)
  p->stats_stage = hc;
}

// ------------------------------------------------------ mutual pair lists
// The mutual near field (Sec. 5, P2Preduce) visits every pair of distinct
// neighbour leaves once, as (a, near[a][s]) for the forward slots
// s = 14..26 (the offsets after the leaf itself in slot order; slot 26 - s
// is the opposite offset).  Launch (s, c) takes the leaves a of colour c:
// the parity of a's grid coordinate along the first non-zero axis of the
// offset.  Along that axis a and its neighbour differ by one, so their
// parities differ, and no leaf is a's side of one pair and the neighbour's
// side of another in the same launch: the launch's pairs touch disjoint
// leaves.  Flag (2k + c) * nl + a marks leaf a in list (14 + k, c).
__global__ void mutual_flags_kernel(const uint64_t* __restrict__ leaf_keys, int bits,
                                    const int* __restrict__ near, int64_t nl,
                                    int* __restrict__ flags) {
  const int64_t a = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (a >= nl) return;
  int c[3];
  demorton3(leaf_keys[a], bits, c);
  for (int k = 0; k < kMutualSlots; ++k) {
    const int s = kMutualFirstSlot + k;
    const int dx = s / 9 - 1, dy = (s / 3) % 3 - 1;
    const int colour = c[dx != 0 ? 0 : dy != 0 ? 1 : 2] & 1;
    const bool has = near[27 * a + s] >= 0;
    flags[(2 * k) * nl + a] = has && colour == 0;
    flags[(2 * k + 1) * nl + a] = has && colour == 1;
  }
}

// list[scan[i]] = leaf of flag i, for the set flags; then the list bounds
__global__ void mutual_emit_kernel(const int* __restrict__ flags, const int64_t* __restrict__ scan,
                                   int64_t nl, int* __restrict__ list) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= 2 * kMutualSlots * nl) return;
  if (flags[i]) list[scan[i]] = int(i % nl);
}

__global__ void mutual_bounds_kernel(const int* __restrict__ flags,
                                     const int64_t* __restrict__ scan, int64_t nl,
                                     int64_t* __restrict__ off) {
  const int k = threadIdx.x;
  const int64_t m = 2 * kMutualSlots * nl;
  if (k < 2 * kMutualSlots) off[k] = scan[k * nl];
  if (k == 2 * kMutualSlots) off[k] = scan[m - 1] + flags[m - 1];
}

__global__ void int_to_i64_kernel(const int* __restrict__ in, int64_t* __restrict__ out,
                                  int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
}

void build_mutual_lists(fmm_plan_s* p, hipStream_t s) {
  const int64_t nl = p->nleaf, m = 2 * kMutualSlots * nl;
  std::vector<void*> tmp;
  struct TmpGuard {
    std::vector<void*>& v;
    hipStream_t s;
    ~TmpGuard() {
      (void)hipStreamSynchronize(s);
      for (void* q : v) dev_free(q);
    }
  } guard{tmp, s};
  auto talloc = [&](size_t b) {
    void* q = dev_alloc(b);
    tmp.push_back(q);
    return q;
  };
  int* flags = static_cast<int*>(talloc(sizeof(int) * m));
  int64_t* scan = static_cast<int64_t*>(talloc(sizeof(int64_t) * m));
  int64_t* off_d = static_cast<int64_t*>(talloc(sizeof(int64_t) * (2 * kMutualSlots + 1)));
  mutual_flags_kernel<<<grid_for(nl, 256), 256, 0, s>>>(p->lev[p->height - 1].keys,
                                                        p->height - 1, p->near, nl, flags);
  FMM_HIP_CHECK(hipGetLastError());
  int_to_i64_kernel<<<grid_for(m, 256), 256, 0, s>>>(flags, scan, m);
  FMM_HIP_CHECK(hipGetLastError());
  exclusive_scan<int64_t>(scan, scan, m, s, tmp);
  mutual_bounds_kernel<<<1, 64, 0, s>>>(flags, scan, nl, off_d);
  FMM_HIP_CHECK(hipGetLastError());
  int64_t off[2 * kMutualSlots + 1];
  FMM_HIP_CHECK(hipMemcpyAsync(off, off_d, sizeof(off), hipMemcpyDeviceToHost, s));
  FMM_HIP_CHECK(hipStreamSynchronize(s));
  const int64_t total = off[2 * kMutualSlots];
  int* list = static_cast<int*>(p->alloc(sizeof(int) * std::max<int64_t>(total, 1)));
  mutual_emit_kernel<<<grid_for(m, 256), 256, 0, s>>>(flags, scan, nl, list);
  FMM_HIP_CHECK(hipGetLastError());
  p->mutual_list = list;
  for (int k = 0; k <= 2 * kMutualSlots; ++k) p->mutual_off[k] = off[k];
}

void plan_stats(fmm_plan_s* p) {
  const unsigned long long* hc = p->stats_stage;
  if (!hc) return;
  for (int k = 0; k < kOffsets; ++k) p->pairs_by_kid[k] = int64_t(hc[kMaxHeight + 2 + k]);
  p->near_pairs = int64_t(hc[kMaxHeight]);
  p->far_pairs = 0;
  for (int l = 0; l < kMaxHeight; ++l) {
    p->far_pairs_level[l] = int64_t(hc[l]);
    p->far_pairs += int64_t(hc[l]);
  }
  p->active_slots = int64_t(hc[kMaxHeight + 1]);
  p->m2l_groups = int64_t(hc[kMaxHeight + 2 + kOffsets]);
  p->m2l_groups_empty = int64_t(hc[kMaxHeight + 3 + kOffsets]);
  // plans whose tiles leave many 16-target groups without a source at an
  // offset (points on surfaces) take the compressed M2L that skips them
  p->m2l_gskip = p->m2l_groups > 0 && 10 * p->m2l_groups_empty >= p->m2l_groups;
  p->stats_stage = nullptr;
}

}  // namespace fmm
