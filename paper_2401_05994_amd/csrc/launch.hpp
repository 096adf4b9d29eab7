// Kernel launches that a batch can regroup (gfx950).
//
// A kernel body is a __device__ function whose first two parameters are the
// block index and the grid size it runs with (G3); the rest are its
// arguments.  Its __global__ entry passes blockIdx and gridDim with its own
// (restrict-qualified) arguments; MG_LAUNCH launches that entry, or, while a
// Recorder is installed on the calling thread, records (body, grid,
// arguments) instead.  A batch records
// the launches of every field and replays them grouped: one k_group launch
// runs the same body for many records, each block finding its record in a
// device table of (first block, grid, arguments) by a binary search over the
// first blocks.  The body's code is the same in both launches.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <type_traits>
#include <utility>
#include <vector>

namespace mg {

struct G3 {
  uint32_t x, y, z;
};

// Arguments of a body as a trivially copyable aggregate.
template <typename... A>
struct Pack;
template <>
struct Pack<> {};
template <typename H, typename... R>
struct Pack<H, R...> {
  H h;
  Pack<R...> r;
};

template <size_t I, typename H, typename... R>
__host__ __device__ inline const auto& pack_get(const Pack<H, R...>& p) {
  if constexpr (I == 0)
    return p.h;
  else
    return pack_get<I - 1>(p.r);
}

template <typename F>
struct BodyArgs;
template <typename... A>
struct BodyArgs<void (*)(G3, G3, A...)> {
  using P = Pack<std::decay_t<A>...>;
  static constexpr size_t N = sizeof...(A);
};

template <auto F, typename P, size_t... I>
__device__ __forceinline__ void body_invoke(G3 b, G3 g, const P& p, std::index_sequence<I...>) {
  F(b, g, pack_get<I>(p)...);
}

template <typename... A, typename... X>
inline Pack<A...> make_pack(const Pack<A...>*, X&&... x) {
  return Pack<A...>{static_cast<A>(x)...};
}

template <auto F>
using PackOf = typename BodyArgs<decltype(F)>::P;

template <typename P>
struct GroupJob {
  uint32_t begin, gx, gy, gz;
  P p;
};

// The record of block b: the last job whose first block is <= b.
template <typename P>
__device__ __forceinline__ const GroupJob<P>& group_find(const GroupJob<P>* jobs, uint32_t njobs, uint32_t b) {
  uint32_t lo = 0, hi = njobs;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (jobs[mid].begin <= b)
      lo = mid;
    else
      hi = mid;
  }
  return jobs[lo];
}

template <auto F, int THREADS>
__global__ void __launch_bounds__(THREADS) k_group(const GroupJob<PackOf<F>>* __restrict__ jobs, uint32_t njobs) {
  const GroupJob<PackOf<F>>& j = group_find(jobs, njobs, blockIdx.x);
  const uint32_t local = blockIdx.x - j.begin;
  body_invoke<F>(G3{local % j.gx, (local / j.gx) % j.gy, local / (j.gx * j.gy)}, G3{j.gx, j.gy, j.gz}, j.p,
                 std::make_index_sequence<BodyArgs<decltype(F)>::N>{});
}

template <auto F, int THREADS, int WPE>
__global__ void __launch_bounds__(THREADS) __attribute__((amdgpu_waves_per_eu(WPE)))
k_group_w(const GroupJob<PackOf<F>>* __restrict__ jobs, uint32_t njobs) {
  const GroupJob<PackOf<F>>& j = group_find(jobs, njobs, blockIdx.x);
  const uint32_t local = blockIdx.x - j.begin;
  body_invoke<F>(G3{local % j.gx, (local / j.gx) % j.gy, local / (j.gx * j.gy)}, G3{j.gx, j.gy, j.gz}, j.p,
                 std::make_index_sequence<BodyArgs<decltype(F)>::N>{});
}

// What a batch needs to regroup the records of one body.
struct GroupOps {
  size_t job_bytes;  // sizeof(GroupJob<P>)
  void (*write_job)(void* dst, uint32_t begin, dim3 grid, const void* pack);
  void (*launch)(const void* d_jobs, uint32_t njobs, uint32_t blocks, hipStream_t st);
};

template <auto F, int THREADS, int WPE>
const GroupOps* group_ops() {
  using P = PackOf<F>;
  static const GroupOps ops{
      sizeof(GroupJob<P>),
      [](void* dst, uint32_t begin, dim3 grid, const void* pack) {
        GroupJob<P> j;
        std::memset(&j, 0, sizeof(j));
        j.begin = begin;
        j.gx = grid.x;
        j.gy = grid.y;
        j.gz = grid.z;
        std::memcpy(&j.p, pack, sizeof(P));
        std::memcpy(dst, &j, sizeof(j));
      },
      [](const void* d_jobs, uint32_t njobs, uint32_t blocks, hipStream_t st) {
        const auto* jobs = static_cast<const GroupJob<P>*>(d_jobs);
        if constexpr (WPE > 0)
          hipLaunchKernelGGL((k_group_w<F, THREADS, WPE>), dim3(blocks), dim3(THREADS), 0, st, jobs, njobs);
        else
          hipLaunchKernelGGL((k_group<F, THREADS>), dim3(blocks), dim3(THREADS), 0, st, jobs, njobs);
      }};
  return &ops;
}

struct LaunchRecord {
  const GroupOps* ops;
  dim3 grid;
  std::vector<uint8_t> pack;
  int phase;
};

// Installed on a thread, it receives the launches MG_LAUNCH records there,
// each tagged with the phase the caller has set (a batch aligns fields phase
// by phase).
struct Recorder {
  std::vector<LaunchRecord> recs;
  int phase = 0;
};
Recorder*& recorder();

// Records (body, grid, arguments) when a Recorder is installed on the calling
// thread (true), else does nothing (false).
template <auto F, int THREADS, int WPE = 0, typename... X>
bool mg_record(dim3 grid, X&&... x) {
  Recorder* r = recorder();
  if (!r) return false;
  using P = PackOf<F>;
  const P p = make_pack(static_cast<const P*>(nullptr), std::forward<X>(x)...);
  LaunchRecord rec{group_ops<F, THREADS, WPE>(), grid, std::vector<uint8_t>(sizeof(P)), r->phase};
  std::memcpy(rec.pack.data(), &p, sizeof(P));
  r->recs.push_back(std::move(rec));
  return true;
}

}  // namespace mg

// A launch of KERNEL, the __global__ entry of BODY (same arguments, its pointer
// parameters declared as the body declares them), or its record while a
// batch records.  Parenthesise BODY, KERNEL and GRID when they hold commas.
#define MG_LAUNCH(BODY, KERNEL, THREADS, WPE, GRID, ST, ...)                                  \
  do {                                                                                        \
    if (!::mg::mg_record<BODY, (THREADS), (WPE)>(GRID, __VA_ARGS__))                          \
      hipLaunchKernelGGL(KERNEL, GRID, dim3(THREADS), 0, ST, __VA_ARGS__);                    \
  } while (0)
