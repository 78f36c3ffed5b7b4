// Stable LSD radix sort of u32 keys carrying one or two u32 values, 8-bit digits, in the
// Onesweep structure (Adinets and Merrill, "Onesweep: A Faster Least
// Significant Digit Radix Sort for GPUs", 2022): the kernels that produce the
// keys build the digit histograms of all passes, then each pass is a single kernel whose
// blocks each rank the keys of one partition locally and resolve the global
// digit offsets with a decoupled look-back over the preceding partitions.
// A block takes its partition index from an atomic ticket when it starts, so
// every partition it waits on belongs to a block that is already running.
// (Block index as partition index is not enough: blocks are dealt to the 8
// XCDs round-robin and each XCD dispatches its share on its own, so with
// other kernels resident a block can start before its predecessor, and two
// look-back kernels can then wait on each other.)
//
// The look-back is two-level: partitions form groups of kGroupParts, and
// the last partition of each group publishes the group's aggregate (from
// per-partition aggregate copies that are never upgraded) and later its
// inclusive prefix.  A block sums its own group's predecessors, then whole
// groups, so it reads at most kGroupParts + ceil(groups / kLookWin) windows
// instead of one window per kLookWin predecessors back to the nearest
// inclusive one, which with hundreds of partitions all starting together
// was a long chain of round trips and a quadratic volume of status reads.
//
// CDNA4 specifics: local ranking is done per 64-lane wavefront with eight
// ballots per item (a match-any on the digit bits); each wave owns a
// contiguous run of the partition so ranks stay stable; look-back status
// words are device-scope relaxed atomics, and every wait is bounded.
#include "octgs_internal.h"

namespace octgs {

namespace {

constexpr uint32_t kFlagAgg = 1u << 30;
constexpr uint32_t kFlagInc = 2u << 30;
constexpr uint32_t kValMask = (1u << 30) - 1;
constexpr int kLookWin = 16;

// Sum, for the status words w(q) = lb[q * stride] with q from p down to lo
// (nearest first), of the values up to and including the nearest inclusive
// word; spins while any word it needs is unpublished.  Returns whether an
// inclusive word was met (otherwise everything down to lo was summed).  A
// wait past the bound sets *err_flag and stops.
__device__ __forceinline__ bool lookback_sum(const uint32_t *lb, size_t stride, int64_t p,
                                             int64_t lo, uint32_t &acc, uint32_t *err_flag) {
  uint32_t spins = 0;
  while (p >= lo) {
    const int cnt = (int)min<int64_t>(kLookWin, p - lo + 1);
    uint32_t v[kLookWin];
#pragma unroll
    for (int i = 0; i < kLookWin; ++i) v[i] = ld_acq(lb + (size_t)(p - min(i, cnt - 1)) * stride);
    bool ready = true, found = false;
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < kLookWin; ++i) {
      if (i < cnt && !found) {
        const uint32_t f = v[i] & ~kValMask;
        ready = ready && f != 0u;
        sum += v[i] & kValMask;
        found = f == kFlagInc;
      }
    }
    if (!ready) {
      if (++spins > kSpinLimit) {
        atomicOr(err_flag, 1u);
        return true;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    acc += sum;
    if (found) return true;
    p -= cnt;
  }
  return false;
}

template <int NV, int PART>
struct PassSmem {
  uint32_t wcnt[4][256];     // per-wave digit counters, then per-wave exclusive offsets
  uint32_t dstart[256];      // local start of each digit in the partition
  uint32_t gbase[256];       // global write base of each digit for this partition
  uint32_t hexcl[256];       // global exclusive prefix of the pass histogram
  uint32_t keys[PART];
  uint32_t vals[NV][PART];
  uint32_t tmp[8];
};

// NV = 1 or 2 value arrays travel with the keys; ITEMS keys per thread, so a
// partition is PART = 256 * ITEMS keys.
template <int NV, int ITEMS>
__global__ __launch_bounds__(kBlock) void k_sort_pass(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin,
    const uint32_t *__restrict__ vin2, uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
    uint32_t *__restrict__ vout2, const uint32_t *__restrict__ count, int shift,
    uint32_t *__restrict__ hist, int hist_copies, uint32_t hist_stride, int fold_passes,
    uint32_t *__restrict__ lookback, uint32_t *__restrict__ groups, uint32_t *__restrict__ ticket,
    uint32_t *__restrict__ err_flag) {
  constexpr int PART = kBlock * ITEMS;
  __shared__ PassSmem<NV, PART> sm;
  __shared__ uint32_t s_part;
  const uint32_t n = *count;
  const uint32_t nparts = (n + PART - 1) / PART;
  const int t = threadIdx.x, w = t / kWave, l = __lane_id();
  const uint64_t lt = lanemask_lt();

  // exactly the first nparts blocks stay, and they take tickets 0..nparts-1
  if (blockIdx.x >= nparts) return;
  if (t == 0) s_part = atomicAdd(ticket, 1u);  // its latency overlaps the histogram scan

  // exclusive scan of the pass histogram (the sum of its copies) over digits
  {
    uint32_t hc[kHistCopies], hv = 0, tot;
#pragma unroll
    for (int c = 0; c < kHistCopies; ++c)
      hc[c] = c < hist_copies ? hist[(size_t)c * hist_stride + t] : 0u;  // all loads in flight
#pragma unroll
    for (int c = 0; c < kHistCopies; ++c) hv += hc[c];
    uint32_t ex = block_excl_scan(hv, sm.tmp, &tot);
    sm.hexcl[t] = ex;
  }

  {
    for (int i = t; i < 4 * 256; i += kBlock) (&sm.wcnt[0][0])[i] = 0u;
    __syncthreads();
    const uint32_t part = s_part;
    const uint32_t base = part * PART;

    // load and rank: wave w owns keys [base + 64 w ITEMS, base + 64 (w + 1) ITEMS)
    uint32_t key[ITEMS], val[ITEMS], val2[ITEMS], rank[ITEMS];
    int dig[ITEMS];
    // unconditional loads at a clamped index keep all of them in flight
    // together; items past the end are masked by dig = -1
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const uint32_t idx = base + w * (kWave * ITEMS) + j * kWave + l;
      key[j] = kin[min(idx, n - 1)];
      val[j] = vin[min(idx, n - 1)];
      if (NV == 2) val2[j] = vin2[min(idx, n - 1)];
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const uint32_t idx = base + w * (kWave * ITEMS) + j * kWave + l;
      dig[j] = idx < n ? (int)((key[j] >> shift) & 255u) : -1;
    }
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      const int d = dig[j];
      uint64_t peers = ballot(d >= 0);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        int bit = (d >> b) & 1;
        uint64_t bal = ballot(bit);
        peers &= bit ? bal : ~bal;
      }
      uint32_t before = 0;
      if (d >= 0) before = sm.wcnt[w][d];
      // all lanes of the wave have read before any leader writes
      __builtin_amdgcn_wave_barrier();
      if (d >= 0) {
        rank[j] = before + (uint32_t)__popcll(peers & lt);
        if ((peers & lt) == 0) sm.wcnt[w][d] = before + (uint32_t)__popcll(peers);
      }
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();

    // thread t owns digit t: per-wave exclusive offsets and the block total
    uint32_t c0 = sm.wcnt[0][t], c1 = sm.wcnt[1][t], c2 = sm.wcnt[2][t], c3 = sm.wcnt[3][t];
    uint32_t tot = c0 + c1 + c2 + c3;
    // status rows: [part][0..255] the digit's aggregate, later its inclusive
    // prefix; [part][256..511] a copy of the aggregate for the group sum
    uint32_t *row = lookback + (size_t)part * kLbRow;
    st_rel(&row[t], (part == 0 ? kFlagInc : kFlagAgg) | tot);
    st_rel(&row[256 + t], kFlagAgg | tot);
    uint32_t blk_tot;
    uint32_t ds = block_excl_scan(tot, sm.tmp, &blk_tot);
    sm.dstart[t] = ds;
    sm.wcnt[0][t] = ds;
    sm.wcnt[1][t] = ds + c0;
    sm.wcnt[2][t] = ds + c0 + c1;
    sm.wcnt[3][t] = ds + c0 + c1 + c2;

    const uint32_t grp = part / kGroupParts;
    const bool closer = part % kGroupParts == kGroupParts - 1;
    if (closer) {
      // the group's aggregate: its partitions' aggregate copies, all running
      uint32_t gs = 0;
      lookback_sum(lookback + 256 + t, kLbRow, part, (int64_t)grp * kGroupParts, gs, err_flag);
      st_rel(&groups[(size_t)grp * 256 + t], kFlagAgg | (gs & kValMask));
    }
    uint32_t excl = 0;
    if (part > 0) {
      // the own group's predecessors, then whole groups
      const bool found = lookback_sum(lookback + t, kLbRow, (int64_t)part - 1,
                                      (int64_t)grp * kGroupParts, excl, err_flag);
      if (!found && grp > 0) lookback_sum(groups + t, 256, (int64_t)grp - 1, 0, excl, err_flag);
      const uint32_t inc = kFlagInc | ((excl + tot) & kValMask);
      st_rel(&row[t], inc);
      if (closer) st_rel(&groups[(size_t)grp * 256 + t], inc);
    }
    sm.gbase[t] = sm.hexcl[t] + excl;
    __syncthreads();

    // place keys in LDS in local sorted order
#pragma unroll
    for (int j = 0; j < ITEMS; ++j) {
      if (dig[j] >= 0) {
        uint32_t pos = sm.wcnt[w][dig[j]] + rank[j];
        sm.keys[pos] = key[j];
        sm.vals[0][pos] = val[j];
        if (NV == 2) sm.vals[NV - 1][pos] = val2[j];
      }
    }
    __syncthreads();
    const uint32_t cnt = min((uint32_t)PART, n - base);
    for (uint32_t i = t; i < cnt; i += kBlock) {
      uint32_t k = sm.keys[i];
      uint32_t d = (k >> shift) & 255u;
      uint32_t dst = sm.gbase[d] + (i - sm.dstart[d]);
      if (dst < n) {  // always true unless a look-back wait hit its bound
        kout[dst] = k;
        vout[dst] = sm.vals[0][i];
        if (NV == 2) vout2[dst] = sm.vals[NV - 1][i];
      }
    }
  }
  // the first pass folds the later passes' histogram copies into copy 0,
  // after its own look-back so the chain does not wait for it; the later
  // passes then read one copy
  if (blockIdx.x == 0) {
    for (int q = 1; q <= fold_passes; ++q) {
      uint32_t hc[kHistCopies], hv = 0;
#pragma unroll
      for (int c = 0; c < kHistCopies; ++c)
        hc[c] = c < hist_copies ? hist[(size_t)c * hist_stride + 256 * q + t] : 0u;
#pragma unroll
      for (int c = 0; c < kHistCopies; ++c) hv += hc[c];
      hist[256 * q + t] = hv;
    }
  }
}

// Pass p of a sort: from buffers p % 2 to the others.
template <int ITEMS>
void launch_pass(uint32_t *keys[2], uint32_t *vals[2], uint32_t *const *vals2,
                 const uint32_t *count, int p, int grid, uint32_t *hist, int copies,
                 uint32_t hist_stride, int fold, uint32_t *lookback, uint32_t *groups,
                 uint32_t *ticket, uint32_t *err_flag, hipStream_t stream) {
  const int src = p & 1, dst = src ^ 1;
  if (vals2)
    hipLaunchKernelGGL((k_sort_pass<2, ITEMS>), dim3(grid), dim3(kBlock), 0, stream, keys[src],
                       vals[src], vals2[src], keys[dst], vals[dst], vals2[dst], count, 8 * p, hist,
                       copies, hist_stride, fold, lookback, groups, ticket, err_flag);
  else
    hipLaunchKernelGGL((k_sort_pass<1, ITEMS>), dim3(grid), dim3(kBlock), 0, stream, keys[src],
                       vals[src], nullptr, keys[dst], vals[dst], nullptr, count, 8 * p, hist,
                       copies, hist_stride, fold, lookback, groups, ticket, err_flag);
}

}  // namespace

hipError_t radix_sort(uint32_t *keys[2], uint32_t *vals[2], uint32_t *const *vals2,
                      const uint32_t *count, int64_t cap, int items, int passes, uint32_t *hist,
                      int hist_copies, uint32_t hist_stride, uint32_t *lookback,
                      uint32_t *tickets, uint32_t *err_flag, hipStream_t stream) {
  if (passes <= 0) return hipSuccess;
  if (hist_copies < 1 || hist_copies > kHistCopies) return hipErrorInvalidValue;
  if (items != kSortItems && items != kTileSortItems) return hipErrorInvalidValue;
  const int64_t part = (int64_t)kBlock * items;
  const int64_t nparts_cap = std::max<int64_t>((cap + part - 1) / part, 1);
  const size_t lb_stride = lookback_pass_words(nparts_cap);
  // one block per possible partition; blocks past the actual count exit
  const int pass_grid = (int)nparts_cap;
  for (int p = 0; p < passes; ++p) {
    const int copies = p == 0 ? hist_copies : 1, fold = p == 0 ? passes - 1 : 0;
    uint32_t *lb = lookback + lb_stride * p;
    uint32_t *groups = lb + (size_t)nparts_cap * kLbRow;
    if (items == kTileSortItems)
      launch_pass<kTileSortItems>(keys, vals, vals2, count, p, pass_grid, hist + 256 * p, copies,
                                  hist_stride, fold, lb, groups, tickets + p, err_flag, stream);
    else
      launch_pass<kSortItems>(keys, vals, vals2, count, p, pass_grid, hist + 256 * p, copies,
                              hist_stride, fold, lb, groups, tickets + p, err_flag, stream);
  }
  return hipGetLastError();
}

}  // namespace octgs
