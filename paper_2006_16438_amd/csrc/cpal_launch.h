// Kernel launches that a batch can regroup stage by stage.
//
// A kernel of the mode update is written as a device body that takes its
// block coordinates (Blk) explicitly, wrapped by a plain __global__ kernel
// that passes the hardware's.  Launchers call launch_b (a body with a batched
// form) or launch_1 (any other kernel).  With no sink installed both launch at
// once; with a sink installed on the calling thread they only describe the
// launch to it: launch_b hands over the arguments as one trivially copyable
// pack and a function that launches the batched kernel k_multi (a launch
// with a 2-D or 3-D grid is handed over as launch_1's is), launch_1 a
// closure that launches the kernel on a given stream.
//
// k_multi runs one body for many independent launches at once: launch d owns
// blocks [pre[d], pre[d+1]) of the grid and reads its arguments from packs[d]
// (device memory); each block finds its launch by binary search over pre and
// runs the body with its index and block count inside that launch.  Every
// launch of one k_multi has the same block size.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <functional>
#include <utility>

namespace cpal {

// Index of a block within its launch and the launch's number of blocks.
struct Blk {
  unsigned x, n;
};
#define CPAL_BLK (::cpal::Blk{blockIdx.x, gridDim.x})

template <size_t I, class T>
struct PackLeaf {
  T v;
};
template <class Seq, class... A>
struct PackImpl;
template <size_t... I, class... A>
struct PackImpl<std::index_sequence<I...>, A...> : PackLeaf<I, A>... {
  __host__ __device__ PackImpl(const A &...a) : PackLeaf<I, A>{a}... {}
  template <class B>
  __device__ __forceinline__ void call(Blk b) const {
    B::run(b, static_cast<const PackLeaf<I, A> &>(*this).v...);
  }
};
// The arguments of one launch, in order.
template <class... A>
using Pack = PackImpl<std::index_sequence_for<A...>, A...>;

template <class B, class P>
__global__ void __launch_bounds__(B::NT, B::MW)
    k_multi(const P *__restrict__ packs, const unsigned *__restrict__ pre, unsigned n) {
  const unsigned bx = blockIdx.x;
  unsigned lo = 0, hi = n;   // pre[lo] <= bx < pre[hi]
  while (hi - lo > 1) {
    const unsigned mid = (lo + hi) >> 1;
    if (pre[mid] <= bx) lo = mid; else hi = mid;
  }
  packs[lo].template call<B>(Blk{bx - pre[lo], pre[lo + 1] - pre[lo]});
}

// Launches k_multi<B, P> over n packs (device memory) with prefix pre.
typedef void (*MultiLaunch)(const void *packs, const unsigned *pre, unsigned n, unsigned blocks,
                            unsigned threads, size_t shmem, hipStream_t s);
template <class B, class P>
void multi_launch(const void *packs, const unsigned *pre, unsigned n, unsigned blocks,
                  unsigned threads, size_t shmem, hipStream_t s) {
  hipLaunchKernelGGL((k_multi<B, P>), dim3(blocks), dim3(threads), shmem, s, (const P *)packs, pre,
                     n);
}

// Receiver of described launches (see above).
struct LaunchSink {
  virtual void batchable(MultiLaunch ml, const void *pack, size_t bytes, size_t align,
                         unsigned grid, unsigned block, size_t shmem) = 0;
  virtual void solo(std::function<void(hipStream_t)> f) = 0;
  virtual ~LaunchSink() = default;
};
// The calling thread's sink (nullptr: launch at once).
LaunchSink *&launch_sink();

// Body struct of a kernel body function FN with a batched form: NT threads
// per block at most, MW waves per SIMD at least (as the plain kernel's bounds).
#define CPAL_BODY(NAME, NTHREADS, MINW, FN)                                      \
  struct NAME {                                                                  \
    static constexpr int NT = NTHREADS, MW = MINW;                               \
    template <class... A>                                                        \
    __device__ __forceinline__ static void run(::cpal::Blk b, const A &...a) {   \
      FN(b, a...);                                                               \
    }                                                                            \
  }

template <class B, class K, class... A>
inline void launch_b(K kern, dim3 g, dim3 blk, size_t shmem, hipStream_t s, const A &...a) {
  LaunchSink *r = launch_sink();
  if (r && g.y == 1 && g.z == 1) {
    const Pack<A...> p(a...);
    r->batchable(&multi_launch<B, Pack<A...>>, &p, sizeof(p), alignof(Pack<A...>), g.x, blk.x,
                 shmem);
    return;
  }
  if (r) {
    r->solo([=](hipStream_t st) { hipLaunchKernelGGL(kern, g, blk, shmem, st, a...); });
    return;
  }
  hipLaunchKernelGGL(kern, g, blk, shmem, s, a...);
}

template <class K, class... A>
inline void launch_1(K kern, dim3 g, dim3 blk, size_t shmem, hipStream_t s, const A &...a) {
  if (LaunchSink *r = launch_sink()) {
    r->solo([=](hipStream_t st) { hipLaunchKernelGGL(kern, g, blk, shmem, st, a...); });
    return;
  }
  hipLaunchKernelGGL(kern, g, blk, shmem, s, a...);
}

}  // namespace cpal
