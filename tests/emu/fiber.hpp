// CPU emulation of one HIP workgroup of 64 or 256 threads (one or four 64-lane wavefronts) with
// cooperative fibers: the threads are ucontext fibers on one host thread that switch round-robin
// at every wave collective (shuffle, ballot, readlane, FP64 matrix-core product) and at every
// workgroup barrier.  Wave collectives are double-buffered by their sequence number, and every lane
// records the source line of the collective it reached: when the lanes of a wave are not all at
// the same collective (a divergent exit from a loop that contains collectives, or a lane that ends
// the kernel while others continue), or the threads of the workgroup are not all at the same
// barrier, the emulator prints the lines and exits with status 9 instead of blocking.  __shared__
// variables become statics (workgroups run one after another).
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
#define __launch_bounds__(...)
#define __shared__ static
#define __restrict__
struct Dim3 { unsigned x = 0, y = 0, z = 0; };

namespace emu {
constexpr int kMaxThreads = 256;
struct Block {
  ucontext_t main_ctx, ctx[kMaxThreads];
  int nthreads = 64;
  int cur = 0;                        // running thread
  bool done[kMaxThreads] = {};
  long long seq[kMaxThreads] = {};    // wave collectives reached per thread
  long long bars[kMaxThreads] = {};   // barriers reached per thread
  int bar_site[kMaxThreads] = {};
  uint64_t slot[2][kMaxThreads];
  double ma[2][kMaxThreads], mb[2][kMaxThreads];
  int site[2][kMaxThreads];
  long long collectives = 0;
};
inline Block* g_blk = nullptr;
inline Dim3 g_block, g_dim, g_grid;
// called before every workgroup starts (a driver poisons the emulated LDS with it: on the GPU a
// workgroup's LDS holds stale values, here statics would otherwise start zeroed)
inline void (*g_block_start)() = nullptr;

[[noreturn]] inline void diverged(const char* what, int a, int sa, int b, int sb) {
  std::fprintf(stderr, "divergence (%s): thread %d at line %d, thread %d at line %d\n", what, a, sa, b, sb);
  std::fflush(stderr);
  std::_Exit(9);
}

// switch to the next thread that has not finished (round-robin)
inline void yield_next() {
  Block& B = *g_blk;
  const int me = B.cur;
  for (int s = 1; s <= B.nthreads; ++s) {
    const int nx = (me + s) % B.nthreads;
    if (B.done[nx]) continue;
    if (nx == me) return;
    B.cur = nx;
    swapcontext(&B.ctx[me], &B.ctx[nx]);
    return;
  }
}

// write this lane's part of wave collective k, yield, check that the whole wave wrote it
inline int wave_arrive(int line, long long& k) {
  Block& B = *g_blk;
  const int me = B.cur;
  k = B.seq[me]++;
  const int b = static_cast<int>(k & 1);
  B.site[b][me] = line;
  if (me == 0) ++B.collectives;
  return b;
}
// A workgroup of fewer than 64 threads is one partial wave: the missing lanes are inactive (they
// take part in no collective, contribute 0 to a ballot and read as 0 through a shuffle).
inline void wave_check(long long k, int b, int line) {
  Block& B = *g_blk;
  const int me = B.cur, w0 = me & ~63;
  const int w1 = w0 + 64 < B.nthreads ? w0 + 64 : B.nthreads;
  for (int l = w0; l < w1; ++l) {
    // lanes earlier in the round may already have gone on (or finished) after this collective
    if (B.seq[l] < k + 1) diverged("lane of the wave finished before this collective", l, B.site[b][l], me, line);
    if (B.site[b][l] != line) diverged("lanes of one wave at different collectives", l, B.site[b][l], me, line);
  }
}

template <class T>
inline T exchange(T v, int src, int line) {
  static_assert(sizeof(T) <= 8, "");
  Block& B = *g_blk;
  long long k;
  const int b = wave_arrive(line, k);
  uint64_t bits = 0;
  std::memcpy(&bits, &v, sizeof(T));
  B.slot[b][B.cur] = bits;
  yield_next();
  wave_check(k, b, line);
  T r{};
  const int s = (B.cur & ~63) + (src & 63);
  if (s < B.nthreads) std::memcpy(&r, &B.slot[b][s], sizeof(T));
  return r;
}
inline unsigned long long ballot(bool p, int line) {
  Block& B = *g_blk;
  long long k;
  const int b = wave_arrive(line, k);
  B.slot[b][B.cur] = p ? 1 : 0;
  yield_next();
  wave_check(k, b, line);
  unsigned long long m = 0;
  const int w0 = B.cur & ~63;
  for (int l = 0; l < 64 && w0 + l < B.nthreads; ++l)
    if (B.slot[b][w0 + l]) m |= 1ull << l;
  return m;
}

typedef double d4 __attribute__((ext_vector_type(4)));
// v_mfma_f64_16x16x4f64: lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
// C/D[l / 16 + 4 r][l % 16], r = 0..3 (the layout measured on gfx950)
inline d4 mfma_f64_16x16x4(double a, double bv, d4 c, int line) {
  Block& B = *g_blk;
  long long k;
  const int b = wave_arrive(line, k);
  B.ma[b][B.cur] = a;
  B.mb[b][B.cur] = bv;
  yield_next();
  wave_check(k, b, line);
  const int w0 = B.cur & ~63, l = B.cur & 63;
  d4 d;
  for (int r = 0; r < 4; ++r) {
    const int i = l / 16 + 4 * r, j = l % 16;
    double acc = c[r];
    for (int p = 0; p < 4; ++p) acc = fma(B.ma[b][w0 + i + 16 * p], B.mb[b][w0 + j + 16 * p], acc);
    d[r] = acc;
  }
  return d;
}

// DPP move (v_mov_b32_dpp) for the controls the device code uses: quad_perm (0x00-0xff), row_mirror
// (0x140), row_half_mirror (0x141), row_bcast:15 (0x142) and row_bcast:31 (0x143).  A lane whose
// row is off in row_mask, or whose source lane does not exist, gets `old` (bound_ctrl off; every
// bank is enabled in the device code).
inline int dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl, int line) {
  Block& B = *g_blk;
  long long k;
  const int b = wave_arrive(line, k);
  B.slot[b][B.cur] = static_cast<uint32_t>(src);
  yield_next();
  wave_check(k, b, line);
  if (bank_mask != 0xf || bound_ctrl) { std::fprintf(stderr, "dpp: unsupported bank_mask/bound_ctrl\n"); std::_Exit(8); }
  const int w0 = B.cur & ~63, l = B.cur & 63, row = l >> 4, lr = l & 15;
  if (!((row_mask >> row) & 1)) return old;
  int s;
  if (ctrl <= 0xff) {
    s = (l & ~3) | ((ctrl >> (2 * (l & 3))) & 3);
  } else if (ctrl == 0x140) {
    s = (l & ~15) | (15 - lr);
  } else if (ctrl == 0x141) {
    s = (l & ~7) | (7 - (l & 7));
  } else if (ctrl == 0x142) {
    if (row == 0) return old;
    s = 16 * (row - 1) + 15;
  } else if (ctrl == 0x143) {
    if (row < 2) return old;
    s = 31;
  } else {
    std::fprintf(stderr, "dpp: unsupported control %#x\n", ctrl);
    std::_Exit(8);
  }
  return static_cast<int>(static_cast<uint32_t>(B.slot[b][w0 + s]));
}

// workgroup barrier: every thread must reach it at the same line
inline void barrier(int line) {
  Block& B = *g_blk;
  const int me = B.cur;
  const long long nb = ++B.bars[me];
  B.bar_site[me] = line;
  while (true) {
    bool all = true;
    for (int t = 0; t < B.nthreads; ++t) {
      if (B.bars[t] >= nb) continue;
      if (B.done[t]) diverged("thread finished while others wait at a barrier", t, -1, me, line);
      all = false;
    }
    if (all) break;
    yield_next();
  }
  for (int t = 0; t < B.nthreads; ++t)
    if (B.bars[t] == nb && B.bar_site[t] != line) diverged("threads at different barriers", t, B.bar_site[t], me, line);
}

template <class F>
inline void thread_entry(unsigned lo, unsigned hi) {
  F* f = reinterpret_cast<F*>((static_cast<uintptr_t>(hi) << 32) | lo);
  (*f)();
  Block& B = *g_blk;
  const int me = B.cur;
  B.done[me] = true;
  // every other lane of the wave must also be finished or finish in this round
  const int w0 = me & ~63;
  for (int l = w0; l < w0 + 64 && l < B.nthreads; ++l)
    if (!B.done[l] && B.seq[l] != B.seq[me]) diverged("lane finished while another is inside a collective", me, -1, l, -1);
  for (int s = 1; s <= B.nthreads; ++s) {
    const int nx = (me + s) % B.nthreads;
    if (!B.done[nx]) {
      B.cur = nx;
      setcontext(&B.ctx[nx]);
    }
  }
  setcontext(&B.main_ctx);
}

// run `kernel` for workgroups 0 .. grid-1 of `threads` threads, one workgroup at a time
template <class F>
inline long long run_grid(unsigned grid, F kernel, int threads = 64) {
  static thread_local char* stacks = nullptr;
  constexpr size_t kStack = 1 << 20;
  if (!stacks) stacks = static_cast<char*>(std::malloc(kStack * kMaxThreads));
  long long total = 0;
  g_grid.x = grid;
  g_dim.x = static_cast<unsigned>(threads);
  for (unsigned blk = 0; blk < grid; ++blk) {
    Block* Bp = new Block();
    Block& B = *Bp;
    B.nthreads = threads;
    g_blk = Bp;
    g_block.x = blk;
    for (int l = 0; l < threads; ++l) {
      getcontext(&B.ctx[l]);
      B.ctx[l].uc_stack.ss_sp = stacks + kStack * l;
      B.ctx[l].uc_stack.ss_size = kStack;
      B.ctx[l].uc_link = nullptr;
      const uintptr_t p = reinterpret_cast<uintptr_t>(&kernel);
      makecontext(&B.ctx[l], reinterpret_cast<void (*)()>(&thread_entry<F>), 2, static_cast<unsigned>(p & 0xffffffffu),
                  static_cast<unsigned>(p >> 32));
    }
    B.cur = 0;
    if (g_block_start) g_block_start();
    swapcontext(&B.main_ctx, &B.ctx[0]);
    for (int l = 0; l < threads; ++l)
      if (!B.done[l]) diverged("thread never finished", l, -1, l, -1);
    total += B.collectives;
    g_blk = nullptr;
    delete Bp;
  }
  return total;
}
}  // namespace emu

inline int __emu_thread() { return emu::g_blk->cur; }
inline int __lane_id() { return emu::g_blk->cur & 63; }
#define threadIdx (Dim3{static_cast<unsigned>(__emu_thread()), 0, 0})
#define blockIdx (emu::g_block)
#define blockDim (emu::g_dim)
#define gridDim (emu::g_grid)
#define __syncthreads() emu::barrier(__LINE__)
#define __shfl_xor(v, off) emu::exchange((v), __lane_id() ^ (off), __LINE__)
#define __shfl(v, src) emu::exchange((v), (src), __LINE__)
#define __builtin_amdgcn_readlane(v, src) emu::exchange<int>((v), (src), __LINE__)
#define __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, x, y, z) emu::mfma_f64_16x16x4((a), (b), (c), __LINE__)
#define __ballot(p) emu::ballot((p), __LINE__)
#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) emu::dpp((old), (src), (ctrl), (rm), (bm), (bc), __LINE__)
#define __builtin_amdgcn_wave_barrier() ((void)emu::exchange<int>(0, 0, __LINE__))
#define __builtin_amdgcn_fence(order, scope) ((void)0)
inline int __ffsll(long long v) { return __builtin_ffsll(v); }
inline int __popcll(unsigned long long v) { return __builtin_popcountll(v); }
template <class T> inline T atomicAdd(T* p, T v) { T o = *p; *p = o + v; return o; }
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
