// CPU emulation of one 64-lane HIP workgroup, to run the generated device source of the
// one-wavefront-per-cell form on the host: 64 threads are the lanes; shuffles, ballots,
// readlane and __syncthreads are collectives over a barrier, so a collective reached by only
// part of the wave deadlocks (the test's time limit reports it) instead of passing silently.
// __shared__ arrays become statics shared by the 64 threads (one workgroup at a time).
#pragma once
#include <atomic>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <algorithm>
using std::exp; using std::log; using std::fma; using std::fabs; using std::sqrt; using std::ldexp; using std::fmax; using std::fmin; using std::log2;
#define __device__
#define __global__
#define __host__
#define __forceinline__ inline
#define __noinline__
#define __launch_bounds__(x)
#define __shared__ static
#define __restrict__
struct Dim3 { unsigned x = 0, y = 0, z = 0; };
extern thread_local Dim3 threadIdx, blockIdx;
extern Dim3 blockDim, gridDim;
extern std::barrier<>* g_bar;
extern thread_local long long g_collectives;
inline int __lane_id() { return (int)(threadIdx.x & 63); }
inline void __syncthreads() { ++g_collectives; g_bar->arrive_and_wait(); }
template <class T> inline T emu_exchange(T v, int src) {
  static T slot[64];
  ++g_collectives;
  slot[__lane_id()] = v; g_bar->arrive_and_wait();
  T r = slot[src & 63]; g_bar->arrive_and_wait();
  return r;
}
inline double __shfl_xor(double v, int off) { return emu_exchange(v, __lane_id() ^ off); }
inline unsigned long long __shfl_xor(unsigned long long v, int off) { return emu_exchange(v, __lane_id() ^ off); }
inline double __shfl(double v, int src) { return emu_exchange(v, src); }
inline unsigned long long __shfl(unsigned long long v, int src) { return emu_exchange(v, src); }
inline int __shfl(int v, int src) { return emu_exchange(v, src); }
inline int __builtin_amdgcn_readlane(int v, int src) { return emu_exchange(v, src); }
inline unsigned long long __ballot(bool p) {
  static std::atomic<unsigned long long> acc; static unsigned long long res;
  ++g_collectives;
  if (__lane_id() == 0) acc = 0; g_bar->arrive_and_wait();
  if (p) acc |= 1ull << __lane_id(); g_bar->arrive_and_wait();
  if (__lane_id() == 0) res = acc.load(); g_bar->arrive_and_wait();
  unsigned long long r = res; g_bar->arrive_and_wait();
  return r;
}
inline int __ffsll(long long v) { return __builtin_ffsll(v); }
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
extern std::mutex g_atomic_mu;
template <class T> inline T atomicAdd(T* p, T v) { std::lock_guard<std::mutex> l(g_atomic_mu); T o = *p; *p = o + v; return o; }
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
