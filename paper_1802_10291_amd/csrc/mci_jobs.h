// mci_jobs.h -- merged launches of an uneven batch.
//
// An uneven batch holds many plans, each with its own sequence of kernel launches.  Instead
// of queueing every plan's launches separately, the batch records them once ("jobs") and
// runs, per step of the sequences, one persistent launch per kernel template: its
// workgroups walk a device table of job descriptors (the argument struct each job's launch
// would have received) and a prefix table of the jobs' workgroup counts, so that one launch
// carries the work of every size class that uses that kernel at that step.  The merged form
// is opt-in (MCI_BATCH_MERGED=1 when the batch is created).
//
// Recording.  While a JobRecorder is installed on the calling thread, the launch helpers of
// the supported kernel families append a Job instead of launching.  The data pointers a job
// holds are then tagged offsets: the batch's input, output and workspace are passed to the
// recorded call as kTagIn, kTagOut and kTagWs (plus any offset the host code adds), and the
// merged kernel adds the pointers of the actual call (JobBases) back.  Plan and batch tables
// (twiddles, apply tables, offset tables) are ordinary device pointers and pass unchanged.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <vector>

namespace mci {

struct JobBases {
  const char* in;
  char* out;
  char* ws;
};

// Device addresses stay below 2^57, so the top bits can carry the tag of a recorded pointer.
constexpr uintptr_t kTagShift = 60;
constexpr uintptr_t kTagIn = (uintptr_t)1 << kTagShift;
constexpr uintptr_t kTagOut = (uintptr_t)2 << kTagShift;
constexpr uintptr_t kTagWs = (uintptr_t)3 << kTagShift;

template <typename T>
__device__ __forceinline__ T* rebase(T* p, const JobBases& b) {
  const uintptr_t v = (uintptr_t)p;
  const uintptr_t tag = v >> kTagShift;
  const uintptr_t off = v & (((uintptr_t)1 << kTagShift) - 1);
  if (tag == 1) return (T*)(b.in + off);
  if (tag == 2) return (T*)(b.out + off);
  if (tag == 3) return (T*)(b.ws + off);
  return p;
}

// The job of virtual workgroup w of a merged launch: the last j with first[j] <= w (first is
// ascending, first[0] = 0, first[n_jobs] = total).  w is uniform over the workgroup, so the
// search runs on scalar loads.
__device__ __forceinline__ int job_of(const int64_t* __restrict__ first, int n_jobs, int64_t w) {
  int lo = 0, hi = n_jobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (first[mid] <= w) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Virtual grid of a job: gx x gy workgroups, numbered x-fastest.
struct JobGrid {
  int64_t gx;
  int gy;
};

// A merged launch: `jobs` (device, n_jobs argument structs of the family), the jobs' grids
// and workgroup prefix (device), `grid` persistent workgroups, `lds` dynamic LDS bytes.
struct MergedLaunch {
  const void* jobs;
  const JobGrid* grids;
  const int64_t* first;
  int n_jobs;
  int64_t total;
  unsigned grid;
  size_t lds;
};
using MergedFn = hipError_t (*)(const MergedLaunch& m, const JobBases& b, hipStream_t s);
// workgroups of the kernel that fit on one CU at the given dynamic LDS (host query)
using OccupancyFn = int (*)(size_t lds);

struct Job {
  MergedFn launch = nullptr;    // the family kernel's merged form for this template (the group key)
  OccupancyFn occupancy = nullptr;
  JobGrid grid{0, 1};
  size_t lds = 0;
  std::vector<unsigned char> args;
};

struct JobRecorder {
  std::vector<Job> jobs;
};

// the recorder installed on the calling thread, or null (launches run normally)
JobRecorder*& job_recorder();

template <typename A>
inline void record_job(MergedFn launch, OccupancyFn occ, const A& args, int64_t gx, int gy, size_t lds) {
  Job j;
  j.launch = launch;
  j.occupancy = occ;
  j.grid = JobGrid{gx, gy};
  j.lds = lds;
  j.args.resize(sizeof(A));
  std::memcpy(j.args.data(), &args, sizeof(A));
  job_recorder()->jobs.push_back(std::move(j));
}

// The body of a merged kernel: every persistent workgroup takes virtual workgroups
// blockIdx.x, blockIdx.x + gridDim.x, ... and runs `fn(args, bx, by, gy)` on each, with a
// barrier between them (the bodies reuse LDS).
template <typename A, typename F>
__device__ __forceinline__ void run_jobs(const A* __restrict__ jobs, const JobGrid* __restrict__ grids,
                                         const int64_t* __restrict__ first, int n_jobs, int64_t total, F fn) {
  for (int64_t w = blockIdx.x; w < total; w += gridDim.x) {
    const int j = job_of(first, n_jobs, w);
    const int64_t v = w - first[j];
    const JobGrid g = grids[j];
    const int by = (int)(v / g.gx);
    const int64_t bx = v - (int64_t)by * g.gx;
    fn(jobs[j], bx, by, g.gy);
    __syncthreads();
  }
}

// Host side of a merged launch of kernel K with NT threads.
template <typename A>
inline hipError_t merged_launch(const void* kernel, unsigned threads, const MergedLaunch& m, const JobBases& b,
                                hipStream_t s) {
  const A* jobs = (const A*)m.jobs;
  const JobGrid* grids = m.grids;
  const int64_t* first = m.first;
  int n_jobs = m.n_jobs;
  int64_t total = m.total;
  JobBases bases = b;
  void* params[] = {(void*)&jobs, (void*)&grids, (void*)&first, (void*)&n_jobs, (void*)&total, (void*)&bases};
  return hipLaunchKernel(kernel, dim3(m.grid), dim3(threads), params, m.lds, s);
}

inline int occupancy_of(const void* kernel, unsigned threads, size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, (int)threads, lds) != hipSuccess) return 1;
  return n > 0 ? n : 1;
}

}  // namespace mci
