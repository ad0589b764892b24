// Gather and scatter between callers' per-job buffers and one contiguous batch.
// A batch of jobs is described by one array of JobSeg records; workgroup b
// serves the job whose block range (from gblk for the gather, sblk for the
// scatter) holds b, found by a wave-uniform binary search, so every workgroup
// copies one contiguous slice of one job.
#include "fdb_internal.hpp"

namespace fdb {

namespace {

constexpr int kBlock = 256;

template <bool GATHER>
__device__ __forceinline__ int seg_of(const JobSeg* __restrict__ seg, int num, int b) {
  int lo = 0, hi = num - 1;  // last job whose first block is <= b
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if ((GATHER ? seg[mid].gblk : seg[mid].sblk) <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// points of job j (n_j x dim floats, row-major) -> batch[off_j * dim ...]
__global__ __launch_bounds__(kBlock) void k_gather(const JobSeg* __restrict__ seg, int num, int dim,
                                                   float* __restrict__ dst) {
  const int j = seg_of<true>(seg, num, blockIdx.x);
  const JobSeg s = seg[j];
  const int64_t len = s.n * dim;
  const int64_t i = static_cast<int64_t>(blockIdx.x - s.gblk) * (kBlock * kSegVec) + threadIdx.x;
  float* out = dst + s.off * dim;
#pragma unroll
  for (int k = 0; k < kSegVec; ++k) {
    const int64_t t = i + k * kBlock;
    if (t < len) out[t] = s.points[t];
  }
}

// batch labels / core flags at [off_j, off_j + n_j) -> job j's own outputs
__global__ __launch_bounds__(kBlock) void k_scatter_jobs(const JobSeg* __restrict__ seg, int num,
                                                         const int32_t* __restrict__ labels,
                                                         const uint8_t* __restrict__ core) {
  const int j = seg_of<false>(seg, num, blockIdx.x);
  const JobSeg s = seg[j];
  const int64_t i = static_cast<int64_t>(blockIdx.x - s.sblk) * (kBlock * kSegVec) + threadIdx.x;
#pragma unroll
  for (int k = 0; k < kSegVec; ++k) {
    const int64_t t = i + k * kBlock;
    if (t < s.n) {
      s.labels[t] = labels[s.off + t];
      if (s.core) s.core[t] = core[s.off + t];
    }
  }
}

}  // namespace

int64_t seg_blocks(int64_t elems) { return ceil_div(elems, static_cast<int64_t>(kBlock) * kSegVec); }

void launch_gather(const JobSeg* seg, int num, int64_t total_blocks, int dim, float* dst, hipStream_t s) {
  if (total_blocks <= 0) return;
  hipLaunchKernelGGL(k_gather, dim3(static_cast<unsigned>(total_blocks)), dim3(kBlock), 0, s, seg, num, dim, dst);
}

void launch_scatter_jobs(const JobSeg* seg, int num, int64_t total_blocks, const int32_t* labels,
                         const uint8_t* core, hipStream_t s) {
  if (total_blocks <= 0) return;
  hipLaunchKernelGGL(k_scatter_jobs, dim3(static_cast<unsigned>(total_blocks)), dim3(kBlock), 0, s, seg, num, labels,
                     core);
}

}  // namespace fdb
