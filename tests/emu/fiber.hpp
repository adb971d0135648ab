// CPU emulation of one 64-lane HIP workgroup with cooperative fibers: the 64 lanes are ucontext
// fibers on one host thread that switch round-robin at every wave collective (shuffle, ballot,
// readlane, barrier).  Each collective is double-buffered by its sequence number, and every lane
// records the source line of the collective it reached: when the lanes of the wave are not all at
// the same collective (a divergent exit from a loop that contains collectives, or a lane that
// ends the kernel while others continue), the emulator prints both lines and exits with status 9
// instead of blocking.  __shared__ arrays become statics (blocks run one after another).
#pragma once
#include <ucontext.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
using std::exp; using std::log; using std::fma; using std::fabs; using std::sqrt; using std::ldexp; using std::fmax;
using std::fmin; using std::log2;
#define __device__
#define __global__
#define __host__
#define __forceinline__ inline
#define __noinline__
#define __launch_bounds__(x)
#define __shared__ static
#define __restrict__
struct Dim3 { unsigned x = 0, y = 0, z = 0; };

namespace emu {
constexpr int kLanes = 64;
struct Wave {
  ucontext_t main_ctx, ctx[kLanes];
  int lane = 0;                 // running lane
  bool done[kLanes] = {};
  long long seq[kLanes] = {};   // collectives reached per lane (at its end, for a finished lane)
  uint64_t slot[2][kLanes];
  int site[2][kLanes];
  long long collectives = 0;
};
inline Wave* g_wave = nullptr;
inline Dim3 g_block, g_dim, g_grid;

[[noreturn]] inline void diverged(const char* what, int a, int sa, int b, int sb) {
  std::fprintf(stderr, "wave divergence (%s): lane %d at line %d, lane %d at line %d\n", what, a, sa, b, sb);
  std::fflush(stderr);
  std::_Exit(9);
}

// switch to the next lane that has not finished (round-robin); a lane that finished while others
// still reach collectives is reported by the caller's check
inline void yield_next() {
  Wave& w = *g_wave;
  const int me = w.lane;
  for (int s = 1; s <= kLanes; ++s) {
    const int nx = (me + s) % kLanes;
    if (w.done[nx]) continue;
    if (nx == me) return;
    w.lane = nx;
    swapcontext(&w.ctx[me], &w.ctx[nx]);
    return;
  }
}

template <class T>
inline T exchange(T v, int src, int line) {
  static_assert(sizeof(T) <= 8, "");
  Wave& w = *g_wave;
  const int me = w.lane;
  const long long k = w.seq[me]++;
  const int b = static_cast<int>(k & 1);
  uint64_t bits = 0;
  std::memcpy(&bits, &v, sizeof(T));
  w.slot[b][me] = bits;
  w.site[b][me] = line;
  if (me == 0) ++w.collectives;
  yield_next();
  // every lane has now written collective k
  for (int l = 0; l < kLanes; ++l) {
    // lanes earlier in this round may already have gone on (or finished) after this collective
    if (w.seq[l] < k + 1) diverged("lane finished before this collective", l, w.site[b][l], me, line);
    if (w.site[b][l] != line) diverged("different collectives", l, w.site[b][l], me, line);
  }
  T r;
  std::memcpy(&r, &w.slot[b][src & 63], sizeof(T));
  return r;
}
inline unsigned long long ballot(bool p, int line) {
  Wave& w = *g_wave;
  const int me = w.lane;
  const long long k = w.seq[me]++;
  const int b = static_cast<int>(k & 1);
  w.slot[b][me] = p ? 1 : 0;
  w.site[b][me] = line;
  yield_next();
  unsigned long long m = 0;
  for (int l = 0; l < kLanes; ++l) {
    if (w.seq[l] < k + 1) diverged("lane finished before this ballot", l, w.site[b][l], me, line);
    if (w.site[b][l] != line) diverged("different collectives", l, w.site[b][l], me, line);
    if (w.slot[b][l]) m |= 1ull << l;
  }
  return m;
}

template <class F>
struct Launch {
  F* f;
};
template <class F>
inline void lane_entry(unsigned lo, unsigned hi) {
  F* f = reinterpret_cast<F*>((static_cast<uintptr_t>(hi) << 32) | lo);
  (*f)();
  Wave& w = *g_wave;
  const int me = w.lane;
  w.done[me] = true;
  // every other lane must also be finished or finish in this round
  for (int l = 0; l < kLanes; ++l)
    if (!w.done[l] && w.seq[l] != w.seq[me]) diverged("lane finished while another is inside a collective", me, -1, l, -1);
  // hand over to the next unfinished lane, or back to the host when all are done
  for (int s = 1; s <= kLanes; ++s) {
    const int nx = (me + s) % kLanes;
    if (!w.done[nx]) {
      w.lane = nx;
      setcontext(&w.ctx[nx]);
    }
  }
  setcontext(&w.main_ctx);
}

// run `kernel` for blocks 0 .. grid-1, one 64-lane block at a time
template <class F>
inline long long run_grid(unsigned grid, F kernel) {
  static thread_local char* stacks = nullptr;
  constexpr size_t kStack = 1 << 20;
  if (!stacks) stacks = static_cast<char*>(std::malloc(kStack * kLanes));
  long long total = 0;
  g_grid.x = grid;
  g_dim.x = kLanes;
  for (unsigned blk = 0; blk < grid; ++blk) {
    Wave w;
    g_wave = &w;
    g_block.x = blk;
    for (int l = 0; l < kLanes; ++l) {
      getcontext(&w.ctx[l]);
      w.ctx[l].uc_stack.ss_sp = stacks + kStack * l;
      w.ctx[l].uc_stack.ss_size = kStack;
      w.ctx[l].uc_link = nullptr;
      const uintptr_t p = reinterpret_cast<uintptr_t>(&kernel);
      makecontext(&w.ctx[l], reinterpret_cast<void (*)()>(&lane_entry<F>), 2, static_cast<unsigned>(p & 0xffffffffu),
                  static_cast<unsigned>(p >> 32));
    }
    w.lane = 0;
    swapcontext(&w.main_ctx, &w.ctx[0]);
    for (int l = 0; l < kLanes; ++l)
      if (!w.done[l]) diverged("lane never finished", l, -1, l, -1);
    total += w.collectives;
    g_wave = nullptr;
  }
  return total;
}
}  // namespace emu

inline int __lane_id() { return emu::g_wave->lane; }
#define threadIdx (Dim3{static_cast<unsigned>(__lane_id()), 0, 0})
#define blockIdx (emu::g_block)
#define blockDim (emu::g_dim)
#define gridDim (emu::g_grid)
#define __syncthreads() ((void)emu::exchange<int>(0, 0, __LINE__))
#define __shfl_xor(v, off) emu::exchange((v), __lane_id() ^ (off), __LINE__)
#define __shfl(v, src) emu::exchange((v), (src), __LINE__)
#define __builtin_amdgcn_readlane(v, src) emu::exchange<int>((v), (src), __LINE__)
#define __ballot(p) emu::ballot((p), __LINE__)
inline int __ffsll(long long v) { return __builtin_ffsll(v); }
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
template <class T> inline T atomicAdd(T* p, T v) { T o = *p; *p = o + v; return o; }
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
