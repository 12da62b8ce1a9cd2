// Batched launches: the workgroups of many independent systems in one grid.
//
// Every kernel of the mixed-precision evaluation is a __device__ body that
// reads its block coordinates from a Wg instead of blockIdx / gridDim.  A
// plain launch runs the body with the hardware coordinates; a batched launch
// runs one grid holding, system after system, each system's whole grid of
// workgroups: workgroup b finds its system by binary search over the
// systems' first workgroups (a descriptor table in device memory) and runs
// the body on that system's argument tuple with its place in that system's
// grid.  A system's evaluation then becomes, per kernel, one slice of a
// launch shared by every system that uses the same kernel instance.
//
// Persistent form: a grid of at most the resident workgroups takes the
// workgroups of the concatenated grid from a device counter, one at a time
// in slice order (systems sorted by cost, largest first: an LPT work queue),
// until all are done; the counter is zeroed by a fill kernel at the head of
// the recording.
//
// Host side: while a LaunchRecorder is installed on the calling thread
// (`launch_recorder()`), the launch functions append each launch (stage,
// batched kernel instance, block size, dynamic LDS, grid, argument tuple) to
// it instead of launching; kpme_batch_evaluate groups the records of all
// systems by stage and kernel instance and launches each group once.
#pragma once
#include <hip/hip_runtime.h>

#include <cstring>
#include <tuple>
#include <utility>
#include <vector>

namespace kpme {

constexpr int kNumXcdB = 8;
__device__ __forceinline__ int xcd_order_b(int b, int n) {
  const int x = b % kNumXcdB, i = b / kNumXcdB;
  const int per = n / kNumXcdB, rem = n % kNumXcdB;
  return x * per + min(x, rem) + i;
}

// A workgroup's coordinates in its system's grid.  hw: the hardware block
// index of a plain launch (kernels then apply their XCD-aware renumbering);
// a batched launch has renumbered its whole grid already.
struct Wg {
  int x, y, z, nx, ny, nz;
  bool hw;
  __device__ static Wg plain() {
    return Wg{static_cast<int>(blockIdx.x), static_cast<int>(blockIdx.y),
              static_cast<int>(blockIdx.z), static_cast<int>(gridDim.x),
              static_cast<int>(gridDim.y), static_cast<int>(gridDim.z), true};
  }
  __device__ int linear() const { return x + nx * (y + ny * z); }
  __device__ int count() const { return nx * ny * nz; }
};

// The XCD-aware logical order of workgroup b of n (see xcd_order) for a
// plain launch; the identity inside a batched one.
__device__ __forceinline__ int wg_order(const Wg& w, int b, int n) {
  return w.hw ? xcd_order_b(b, n) : b;
}

// One system's slice of a batched grid: its first workgroup and its own
// grid extents.  The table holds one more entry whose `first` is the total.
struct BatchSlice {
  int first;
  int nx, ny, nz;
};

// Workgroup b of the concatenated grid: its system by binary search over
// the slices, its coordinates in that system's grid, and the body on that
// system's argument tuple.
template <auto Body, typename... A>
__device__ __forceinline__ void batched_item(const void* args, const BatchSlice* sl, int nsys,
                                             int b) {
  int lo = 0, hi = nsys - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sl[mid].first <= b) lo = mid; else hi = mid - 1;
  }
  const BatchSlice s = sl[lo];
  int r = b - s.first;
  Wg w;
  w.nx = s.nx;
  w.ny = s.ny;
  w.nz = s.nz;
  w.x = r % s.nx;
  r /= s.nx;
  w.y = r % s.ny;
  w.z = r / s.ny;
  w.hw = false;
  const std::tuple<A...>& t = static_cast<const std::tuple<A...>*>(args)[lo];
  std::apply([&](auto... a) { Body(a..., w); }, t);
}

template <auto Body, typename... A>
__device__ __forceinline__ void batched_run(const void* args, const BatchSlice* sl, int nsys) {
  // hardware order: consecutive workgroups go to the XCDs in turn, so every
  // system's slice is spread over the whole chip (grouping slices by XCD
  // measured 10% slower on the 64-system batch: the per-workgroup cost
  // differs between systems and the XCDs finish unevenly)
  batched_item<Body, A...>(args, sl, nsys, static_cast<int>(blockIdx.x));
}

// The persistent loop: thread 0 takes the next item from the queue while the
// current one runs; barriers keep the body's LDS and the broadcast slot from
// being reused before every thread is done with them.
template <auto Body, typename... A>
__device__ __forceinline__ void batched_run_queue(const void* args, const BatchSlice* sl,
                                                  int nsys, int total, int* queue) {
  __shared__ int item;
  int next = 0;
  if (threadIdx.x == 0) next = atomicAdd(queue, 1);
  for (;;) {
    if (threadIdx.x == 0) item = next;
    __syncthreads();
    const int b = item;
    __syncthreads();
    if (b >= total) return;
    if (threadIdx.x == 0) next = atomicAdd(queue, 1);
    batched_item<Body, A...>(args, sl, nsys, b);
  }
}

template <int NT, auto Body, typename... A>
__global__ __launch_bounds__(NT) void batched_kernel(const void* args, const BatchSlice* sl,
                                                     int nsys) {
  batched_run<Body, A...>(args, sl, nsys);
}

// The same with a minimum waves-per-SIMD hint W (kernels that use it).
template <int NT, int W, auto Body, typename... A>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(W))) void batched_kernel_w(
    const void* args, const BatchSlice* sl, int nsys) {
  batched_run<Body, A...>(args, sl, nsys);
}

// Persistent forms of the two.
template <int NT, auto Body, typename... A>
__global__ __launch_bounds__(NT) void batched_kernel_q(const void* args, const BatchSlice* sl,
                                                       int nsys, int total, int* queue) {
  batched_run_queue<Body, A...>(args, sl, nsys, total, queue);
}

template <int NT, int W, auto Body, typename... A>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(W))) void batched_kernel_wq(
    const void* args, const BatchSlice* sl, int nsys, int total, int* queue) {
  batched_run_queue<Body, A...>(args, sl, nsys, total, queue);
}

// Stages of one evaluation, in launch order (a system's launches carry
// strictly increasing stages).
enum LaunchStage {
  LS_BIN_COUNT = 10,
  LS_BIN_SCAN = 11,
  LS_BIN_SCATTER = 12,
  LS_SPREAD = 20,
  LS_COMBINE = 21,
  LS_GRID_SUM = 30,
  LS_STAGE1 = 31,
  LS_STAGE2 = 32,
  LS_FINALIZE = 33,
  LS_GATHER = 40,
};

struct LaunchRecord {
  int stage;
  const void* kernel;   // batched kernel instance (groups records)
  const void* kernel_q; // its persistent form
  int threads;
  size_t lds;
  int nx, ny, nz;
  size_t tuple_size;
  std::vector<unsigned char> args;  // the argument tuple's bytes
};

struct LaunchRecorder {
  std::vector<LaunchRecord> recs;
  bool unsupported = false;  // a launch that has no batched form was reached
};

// The calling thread's recorder (nullptr: launch normally).
LaunchRecorder*& launch_recorder();

// Launch `plain` (the kernel wrapping Body) with args, or record the launch
// for a batched one.  A... are the body's parameter types before its Wg.
template <int NT, auto Body, typename K, typename... A>
hipError_t launch_or_record(int stage, K plain, dim3 grid, size_t lds, hipStream_t st,
                            A... args) {
  if (LaunchRecorder* r = launch_recorder()) {
    if (grid.x == 0 || grid.y == 0 || grid.z == 0) return hipSuccess;
    LaunchRecord rec;
    rec.stage = stage;
    rec.kernel = reinterpret_cast<const void*>(&batched_kernel<NT, Body, A...>);
    rec.kernel_q = reinterpret_cast<const void*>(&batched_kernel_q<NT, Body, A...>);
    rec.threads = NT;
    rec.lds = lds;
    rec.nx = static_cast<int>(grid.x);
    rec.ny = static_cast<int>(grid.y);
    rec.nz = static_cast<int>(grid.z);
    const std::tuple<A...> t(args...);
    rec.tuple_size = sizeof(t);
    rec.args.resize(sizeof(t));
    std::memcpy(rec.args.data(), &t, sizeof(t));
    r->recs.push_back(std::move(rec));
    return hipSuccess;
  }
  hipLaunchKernelGGL(plain, grid, dim3(NT), lds, st, args...);
  return hipGetLastError();
}

// The same for kernels with a waves-per-SIMD hint.
template <int NT, int W, auto Body, typename K, typename... A>
hipError_t launch_or_record_w(int stage, K plain, dim3 grid, size_t lds, hipStream_t st,
                              A... args) {
  if (LaunchRecorder* r = launch_recorder()) {
    if (grid.x == 0 || grid.y == 0 || grid.z == 0) return hipSuccess;
    LaunchRecord rec;
    rec.stage = stage;
    rec.kernel = reinterpret_cast<const void*>(&batched_kernel_w<NT, W, Body, A...>);
    rec.kernel_q = reinterpret_cast<const void*>(&batched_kernel_wq<NT, W, Body, A...>);
    rec.threads = NT;
    rec.lds = lds;
    rec.nx = static_cast<int>(grid.x);
    rec.ny = static_cast<int>(grid.y);
    rec.nz = static_cast<int>(grid.z);
    const std::tuple<A...> t(args...);
    rec.tuple_size = sizeof(t);
    rec.args.resize(sizeof(t));
    std::memcpy(rec.args.data(), &t, sizeof(t));
    r->recs.push_back(std::move(rec));
    return hipSuccess;
  }
  hipLaunchKernelGGL(plain, grid, dim3(NT), lds, st, args...);
  return hipGetLastError();
}

// The batched kernel instance that launch_or_record_w would record for these
// argument types (for setting its attributes).
template <int NT, int W, auto Body, typename... A>
const void* batched_kernel_w_of(A...) {
  return reinterpret_cast<const void*>(&batched_kernel_w<NT, W, Body, A...>);
}
template <int NT, int W, auto Body, typename... A>
const void* batched_kernel_wq_of(A...) {
  return reinterpret_cast<const void*>(&batched_kernel_wq<NT, W, Body, A...>);
}

// Marks the recorder when a launch without a batched form is reached.
inline bool record_unsupported() {
  if (LaunchRecorder* r = launch_recorder()) {
    r->unsupported = true;
    return true;
  }
  return false;
}

// Raises the dynamic-LDS limit of a batched kernel instance.
hipError_t batched_set_lds(const void* kernel, size_t bytes);

}  // namespace kpme
