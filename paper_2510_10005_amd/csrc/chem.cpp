// libchem.so: C ABI (include/chem.h) over per-mechanism generated HIP kernels for gfx950.
#include "chem.h"

#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <memory>
#include <mutex>
#include <sstream>
#include <stdexcept>
#include <string>
#include <thread>
#include <vector>

#include "mechanism.hpp"
#include "noalloc.hpp"

namespace {

thread_local std::string g_last_error;

chem_err fail(chem_err e, const std::string& msg) {
  g_last_error = msg;
  return e;
}

#define HIP_TRY(expr)                                                                       \
  do {                                                                                      \
    hipError_t _e = (expr);                                                                 \
    if (_e != hipSuccess)                                                                   \
      return fail(CHEM_EDEVICE, std::string(#expr) + ": " + hipGetErrorString(_e));         \
  } while (0)

// Registers per lane beyond which the per-cell matrix lives in a device-memory workspace.
constexpr int kDenseLimit = 24;  // n <= 24: one cell per lane, Jacobian and LU in registers
constexpr int kWaveApiLimit = 64;  // 24 < n <= 64: API kernels with one cell per wavefront
constexpr int kBlockLimit = 160;   // n > 24: integrators with one cell per 256-thread workgroup
constexpr int kBlockThreads = 256;
constexpr int kMaxBlock = 256;

const char* kKernelNames[] = {
    "chem_k_thermo",        "chem_k_source",           "chem_k_jacobian",         "chem_k_state_from_TPY",
    "chem_k_mass_fractions", "chem_k_state_from_TPY_vjp", "chem_k_mass_fractions_vjp", "chem_k_fill_u64",
    "chem_k_ros2_persistent", "chem_k_ros2_init",       "chem_k_ros2_step",        "chem_k_be_persistent",
    "chem_k_be_init",       "chem_k_be_step",          "chem_k_be_adjoint",       "chem_k_reduce_blocks",
    "chem_k_sched_scan",    "chem_k_sched_scatter",    "chem_k_jac_transpose",    "chem_k_ros2_persistent_rec",
    "chem_k_ros2_adjoint",  "chem_k_sdirk2_persistent", "chem_k_sdirk4_persistent",
    "chem_k_yass_persistent", "chem_k_T_from_energy", "chem_k_cfd_source", "chem_k_ros2_persistent_lup",
    "chem_k_be_persistent_lup"};
enum KernelId {
  K_THERMO, K_SOURCE, K_JACOBIAN, K_TPY, K_MASSFRAC, K_TPY_VJP, K_MASSFRAC_VJP, K_FILL_U64,
  K_ROS2_PERSISTENT, K_ROS2_INIT, K_ROS2_STEP, K_BE_PERSISTENT, K_BE_INIT, K_BE_STEP, K_BE_ADJOINT,
  K_REDUCE_BLOCKS, K_SCHED_SCAN, K_SCHED_SCATTER, K_JAC_TRANSPOSE, K_ROS2_PERSISTENT_REC, K_ROS2_ADJOINT,
  K_SDIRK2_PERSISTENT, K_SDIRK4_PERSISTENT, K_YASS_PERSISTENT, K_T_FROM_ENERGY, K_CFD_SOURCE,
  K_ROS2_PERSISTENT_LUP, K_BE_PERSISTENT_LUP, K_COUNT
};
// kernels of LU strategy 1 (block form with the factors in LDS only)
bool lu_strategy_kernel(int k) { return k == K_ROS2_PERSISTENT_LUP || k == K_BE_PERSISTENT_LUP; }
// kernels that only the register-resident form (n <= kDenseLimit) has
bool dense_only(int k) {
  return k == K_ROS2_PERSISTENT_REC || k == K_ROS2_ADJOINT || k == K_SDIRK2_PERSISTENT || k == K_SDIRK4_PERSISTENT ||
         k == K_YASS_PERSISTENT;
}
// persistent integration kernel of a method
bool known_method(int m) { return m >= CHEM_BE && m <= CHEM_YASS; }
// fixed-step methods with only the persistent form and no adjoint tape
bool persistent_only(int m) { return m == CHEM_SDIRK2 || m == CHEM_SDIRK4 || m == CHEM_YASS; }
const char* method_name(int m) {
  static const char* names[] = {"backward Euler", "Rosenbrock", "SDIRK-2", "SDIRK-4", "YASS"};
  return known_method(m) ? names[m] : "?";
}
KernelId persistent_kernel(int method) {
  switch (method) {
    case CHEM_ROS2: return K_ROS2_PERSISTENT;
    case CHEM_SDIRK2: return K_SDIRK2_PERSISTENT;
    case CHEM_SDIRK4: return K_SDIRK4_PERSISTENT;
    case CHEM_YASS: return K_YASS_PERSISTENT;
    default: return K_BE_PERSISTENT;
  }
}
constexpr int kSchedBins = 256;  // CHEM_SCHED_BINS in the device code

struct DevChemOpts {  // layout mirrors ChemOpts in the generated source
  double dt, rtol, atol, h_min;
  double newton_rtol, newton_atol_T, newton_atol_Y;
  int n_steps, max_steps, newton_max, halving_max_depth, energy, ckpt_every;
};
struct DevYassOpts {  // layout mirrors YassOpts in the generated source
  double alpha, krylov_rtol;
  int linear_solver, krylov_dim, krylov_max_iter, krylov_precond;
};

uint64_t fnv1a(const std::string& s, uint64_t h = 1469598103934665603ull) {
  for (unsigned char c : s) {
    h ^= c;
    h *= 1099511628211ull;
  }
  return h;
}

std::string default_cache_dir() {
  const char* env = std::getenv("CHEM_KERNEL_CACHE");
  if (env && *env) return env;
  return "/tmp/chem_kernel_cache_" + std::to_string(static_cast<long>(getuid()));
}

void mkdirs(const std::string& path) {
  std::string cur;
  for (size_t i = 0; i < path.size(); ++i) {
    cur += path[i];
    if (path[i] == '/' || i + 1 == path.size()) mkdir(cur.c_str(), 0755);
  }
}

bool read_file(const std::string& p, std::string& out) {
  std::ifstream f(p, std::ios::binary);
  if (!f) return false;
  std::ostringstream ss;
  ss << f.rdbuf();
  out = ss.str();
  return true;
}

std::vector<std::string> compile_options(const std::string& arch) {
  // -fno-signed-zeros: the sign of a zero is never observed on this path (temperatures are tested
  // with > 0, states with isfinite); it lets the compiler drop +0.0 terms and frees registers.
  std::vector<std::string> o = {"--offload-arch=" + arch, "-O3", "-std=c++17", "-fno-signed-zeros", "-Xclang",
                                "-target-feature", "-Xclang", "-packed-fp32-ops"};
  // extra hipRTC flags (e.g. scheduler selection) for tuning experiments; part of the cache key
  if (const char* extra = std::getenv("CHEM_HIPRTC_FLAGS")) {
    std::istringstream ss(extra);
    std::string tok;
    while (ss >> tok) o.push_back(tok);
  }
  return o;
}

// Kernel groups (CHEM_IN_GROUP in the device code).  A register-resident mechanism is one program;
// a larger one is split into one program per group, compiled concurrently, because its code is
// large enough that a single compile is slow.
constexpr int kGroups = 4;
const int kKernelGroup[K_COUNT] = {0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 2, 2, 2, 3, 0, 1, 1, 0, 1, 3, 2, 2, 2, 0, 0, 1, 2};

struct CodeObject {
  std::string code, path;
  chem_err err = CHEM_OK;
  std::string msg;
};

// compile one program (group < 0: all kernels), or fetch it from the cache
void build_one(const std::string& src, const std::string& arch, const std::string& cache_dir, int group,
               CodeObject& out) {
  auto opts = compile_options(arch);
  if (group >= 0) opts.push_back("-DCHEM_KGROUP=" + std::to_string(group));
  int rtc_major = 0, rtc_minor = 0;
  hiprtcVersion(&rtc_major, &rtc_minor);
  std::string key = src + "|" + std::to_string(rtc_major) + "." + std::to_string(rtc_minor);
  for (auto& o : opts) key += "|" + o;
  char name[64];
  std::snprintf(name, sizeof(name), "chem_%016llx.hsaco", static_cast<unsigned long long>(fnv1a(key)));
  out.path = cache_dir + "/" + name;
  if (read_file(out.path, out.code) && !out.code.empty()) return;
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "chem_mechanism.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
    out.err = CHEM_ECOMPILE;
    out.msg = "hiprtcCreateProgram failed";
    return;
  }
  std::vector<const char*> copts;
  for (auto& o : opts) copts.push_back(o.c_str());
  hiprtcResult rc = hiprtcCompileProgram(prog, static_cast<int>(copts.size()), copts.data());
  if (rc != HIPRTC_SUCCESS) {
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    std::string log(ls, '\0');
    if (ls) hiprtcGetProgramLog(prog, &log[0]);
    hiprtcDestroyProgram(&prog);
    if (log.size() > 4000) log = log.substr(0, 4000) + "...";
    out.err = CHEM_ECOMPILE;
    out.msg = "hipRTC compile failed: " + log;
    return;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  out.code.assign(cs, '\0');
  hiprtcGetCode(prog, &out.code[0]);
  hiprtcDestroyProgram(&prog);
  mkdirs(cache_dir);
  const std::string tmp = out.path + ".tmp" + std::to_string(static_cast<long>(getpid())) + "_" +
                          std::to_string(group + 1);
  {
    std::ofstream f(tmp, std::ios::binary);
    f.write(out.code.data(), static_cast<std::streamsize>(out.code.size()));
  }
  std::rename(tmp.c_str(), out.path.c_str());
}

// generate + compile (or fetch from the cache) the code objects of a mechanism: one entry for a
// register-resident mechanism, kGroups entries otherwise.  full_system (register-resident
// mechanisms): the build whose integrators solve for every species, groups 1 (Rosenbrock), 2
// (backward Euler, SDIRK, YASS) and 3 (adjoints) only.
chem_err build_code_objects(const chem::Mechanism& m, const std::string& arch, const std::string& cache_dir,
                            std::vector<CodeObject>& objs, bool full_system = false) {
  const std::string src = chem::generate_source(m, kDenseLimit, full_system);
  const bool split = m.n() > kDenseLimit;
  std::vector<int> groups;
  if (full_system)
    groups = {1, 2, 3};
  else if (split)
    for (int g = 0; g < kGroups; ++g) groups.push_back(g);
  else
    groups = {-1};
  objs.assign(groups.size(), CodeObject{});
  std::vector<std::thread> th;
  for (size_t i = 0; i < groups.size(); ++i)
    th.emplace_back([&, i] { build_one(src, arch, cache_dir, groups[i], objs[i]); });
  for (auto& t : th) t.join();
  for (auto& o : objs)
    if (o.err) return fail(o.err, o.msg);
  return CHEM_OK;
}

chem_err parse_file(const char* path, chem::Mechanism& m) {
  if (!path) return fail(CHEM_EINVAL, "null mechanism path");
  std::string text;
  if (!read_file(path, text)) return fail(CHEM_EPARSE, std::string("cannot read ") + path);
  try {
    m = chem::parse_mechanism(text);
  } catch (const std::exception& e) {
    return fail(CHEM_EPARSE, std::string(path) + ": " + e.what());
  }
  if (m.n() > kBlockLimit)
    return fail(CHEM_EUNSUPPORTED, std::string(path) + ": " + std::to_string(m.ns()) +
                                       " species; at most " + std::to_string(kBlockLimit - 1) + " are supported");
  return CHEM_OK;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  chem_err ensure(size_t b) {
    if (b <= bytes) return CHEM_OK;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    if (hipMalloc(&p, b) != hipSuccess) return fail(CHEM_ENOMEM, "device allocation of " + std::to_string(b) + " bytes failed");
    bytes = b;
    return CHEM_OK;
  }
  template <class T>
  T* as() const { return static_cast<T*>(p); }
};

}  // namespace

struct chem_tape {
  const chem_mech* mech = nullptr;
  int method = CHEM_BE;  // integrator the tape records
  int64_t n_cells = 0;
  int64_t ld = 0;
  int ckpt_every = 1;
  int max_steps = 0;     // Rosenbrock: accepted steps recorded per cell
  bool recorded = false;
  DevChemOpts opts{};
  DevBuf ckpt, nsub, status, hs, nacc;
  int ckpt_slots = 0, nsub_steps = 0;
};

struct chem_mech {
  chem::Mechanism m;
  int n_active = 0;  // T plus the species with a non-zero net coefficient (size of the solved system)
  int device = 0;
  int num_cu = 0;
  std::string arch;
  std::vector<hipModule_t> modules;
  hipFunction_t fn[K_COUNT] = {};
  // full-system build of a register-resident mechanism (integrators in the reactor energy mode),
  // loaded on first use (under mu)
  std::vector<hipModule_t> modules_full;
  hipFunction_t fn_full[K_COUNT] = {};
  bool full_loaded = false;
  std::string cache_dir;
  bool dense = true;
  bool wave = false;      // n > 24: table-driven evaluation; integrators one cell per 256-thread workgroup
  bool wave_api = false;  // 24 < n <= 64: Jacobian API kernel one cell per 64-lane wavefront
  int np = 0;             // padded matrix size of the block form (multiple of 16)
  DevBuf lnA_default, queue, ws, wst, counters_internal, running, seg, gws, gpart, sched, order, jstage;
  unsigned int* running_host = nullptr;
  int launch_block[5][2] = {};  // [method][form]
  int lu_strategy[5] = {};      // [method]: 0 default, 1 LDS-panel LU (block form, factors in LDS)
  int launch_grid[5][2] = {};
  size_t max_shmem = 0;         // LDS bytes one block may use on this device
  // The workspaces above are shared by every stream: each call that uses them records `fence` on
  // its stream, and a call on another stream first waits for it (see StreamFence).
  hipEvent_t fence = nullptr;
  hipStream_t fence_stream = nullptr;
  bool fence_set = false;
  unsigned char* scratch = nullptr;  // this device's scratch array of chem_integrate_noalloc
  std::mutex mu;
  ~chem_mech() {
    if (fence) (void)hipEventDestroy(fence);
    if (running_host) (void)hipHostFree(running_host);
    for (hipModule_t md : modules) (void)hipModuleUnload(md);
    for (hipModule_t md : modules_full) (void)hipModuleUnload(md);
  }
};

namespace {

// The build the calling thread's current integration uses: the full-system one (reactor energy
// mode of a register-resident mechanism) or the regular one.  Per thread, so that calls on other
// threads are not affected; set by FullSystemScope.
thread_local bool t_full_system = false;

struct FullSystemScope {
  bool prev;
  explicit FullSystemScope(bool on) : prev(t_full_system) { t_full_system = on; }
  ~FullSystemScope() { t_full_system = prev; }
};

hipFunction_t kernel_fn(const chem_mech* M, KernelId k) { return t_full_system ? M->fn_full[k] : M->fn[k]; }

// size of the system the integrators solve: T and the reacting species, or every component
int solved_size(const chem_mech* M) { return t_full_system ? M->m.n() : M->n_active; }

chem_err launch(const chem_mech* M, KernelId k, unsigned grid, unsigned block, hipStream_t s, void** args,
                unsigned shmem = 0) {
  if (grid == 0) return CHEM_OK;
  hipError_t e = hipModuleLaunchKernel(kernel_fn(M, k), grid, 1, 1, block, 1, 1, shmem, s, args, nullptr);
  if (e != hipSuccess) return fail(CHEM_EDEVICE, std::string("launch of ") + kKernelNames[k] + ": " + hipGetErrorString(e));
  return CHEM_OK;
}

chem_err launch2d(const chem_mech* M, KernelId k, unsigned gx, unsigned gy, unsigned block, hipStream_t s,
                  void** args) {
  if (gx == 0 || gy == 0) return CHEM_OK;
  hipError_t e = hipModuleLaunchKernel(kernel_fn(M, k), gx, gy, 1, block, 1, 1, 0, s, args, nullptr);
  if (e != hipSuccess) return fail(CHEM_EDEVICE, std::string("launch of ") + kKernelNames[k] + ": " + hipGetErrorString(e));
  return CHEM_OK;
}

unsigned blocks_for(int64_t n, int block) { return static_cast<unsigned>((n + block - 1) / block); }

// Orders a workspace-using call after the previous one on the same mechanism when the two were
// enqueued on different streams; held under chem_mech::mu.  While the stream is being captured
// into a graph nothing is waited on or recorded (the captured work is ordered by its replays).
struct StreamFence {
  chem_mech* M;
  hipStream_t s;
  bool capturing = false, armed = false;
  StreamFence(chem_mech* m, hipStream_t st) : M(m), s(st) {}
  chem_err begin() {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cs));
    capturing = cs != hipStreamCaptureStatusNone;
    if (!capturing && M->fence_set && M->fence_stream != s) HIP_TRY(hipStreamWaitEvent(s, M->fence, 0));
    armed = true;
    return CHEM_OK;
  }
  ~StreamFence() {
    if (!armed || capturing) return;
    if (hipEventRecord(M->fence, s) == hipSuccess) {
      M->fence_stream = s;
      M->fence_set = true;
    }
  }
};

chem_err check_cells(int64_t n_cells, int64_t ld) {
  if (n_cells < 0) return fail(CHEM_EINVAL, "n_cells must be >= 0");
  if (ld < n_cells) return fail(CHEM_EINVAL, "ld must be >= n_cells");
  if (n_cells > (int64_t(1) << 40)) return fail(CHEM_EINVAL, "n_cells too large");
  return CHEM_OK;
}

// the one-wave-per-cell form launches a block per cell (grid limit)
chem_err check_cells(const chem_mech* M, int64_t n_cells, int64_t ld) {
  if (chem_err e = check_cells(n_cells, ld)) return e;
  if (M->wave && n_cells > int64_t(0x7fffffff)) return fail(CHEM_EINVAL, "n_cells must be < 2^31 for this mechanism");
  return CHEM_OK;
}


DevChemOpts to_dev(const chem_integrator_opts& o, int ckpt_every) {
  DevChemOpts d{};
  d.dt = o.dt;
  d.rtol = o.rtol;
  d.atol = o.atol;
  d.h_min = o.h_min;
  d.newton_rtol = o.newton_rtol;
  d.newton_atol_T = o.newton_atol_T;
  d.newton_atol_Y = o.newton_atol_Y;
  d.n_steps = (o.method != CHEM_ROS2 && o.n_steps < 1) ? 1 : o.n_steps;
  d.max_steps = o.max_steps;
  d.newton_max = o.newton_max;
  d.halving_max_depth = o.halving_max_depth;
  d.energy = o.energy;
  d.ckpt_every = ckpt_every > 0 ? ckpt_every : 1;
  return d;
}

DevYassOpts yass_to_dev(const chem_integrator_opts& o) {
  DevYassOpts d{};
  d.alpha = o.yass_alpha;
  d.krylov_rtol = o.krylov_rtol;
  d.linear_solver = o.linear_solver;
  d.krylov_dim = o.krylov_dim;
  d.krylov_max_iter = o.krylov_max_iter;
  d.krylov_precond = o.krylov_precond;
  return d;
}

bool known_energy(int e) { return e == CHEM_CONST_P || e == CHEM_CONST_V || e == CHEM_CONST_P_REACTOR; }

// The reactor form changes every concentration (the density follows T and the mole number), so it
// needs integrators that solve the full system: the block form's (n > 24) and, for register-resident
// mechanisms, those of the full-system build.  Tapes: the backward-Euler adjoints carry the
// dilatation terms (block form; full-system build of the register form); the Rosenbrock adjoint's
// vector-Jacobian products do not.
chem_err check_reactor(const chem_mech* M, const chem_integrator_opts* o, bool tape) {
  (void)M;
  if (o->energy != CHEM_CONST_P_REACTOR) return CHEM_OK;
  if (tape && o->method != CHEM_BE)
    return fail(CHEM_EUNSUPPORTED, "in the constant-pressure reactor form only the backward-Euler adjoint "
                "records a tape");
  return CHEM_OK;
}

chem_err validate_opts(const chem_integrator_opts* o) {
  if (!o) return fail(CHEM_EINVAL, "null options");
  if (!known_method(o->method))
    return fail(CHEM_EINVAL, "unknown method");
  if (!known_energy(o->energy)) return fail(CHEM_EINVAL, "unknown energy mode");
  if (o->form != CHEM_PERSISTENT && o->form != CHEM_PLAIN) return fail(CHEM_EINVAL, "unknown form");
  if (!(o->dt > 0.0) || !std::isfinite(o->dt)) return fail(CHEM_EINVAL, "dt must be positive and finite");
  if (o->n_steps < 0) return fail(CHEM_EINVAL, "n_steps must be >= 0");
  if (o->max_steps < 1) return fail(CHEM_EINVAL, "max_steps must be >= 1");
  if (o->method == CHEM_ROS2 && (!(o->rtol > 0.0) || !(o->atol > 0.0))) return fail(CHEM_EINVAL, "rtol and atol must be positive");
  if (!(o->h_min >= 0.0)) return fail(CHEM_EINVAL, "h_min must be >= 0");
  if (o->newton_max < 1 || o->halving_max_depth < 0 || o->halving_max_depth > 30)
    return fail(CHEM_EINVAL, "newton_max >= 1 and 0 <= halving_max_depth <= 30 required");
  if (o->probe_attempts < 0) return fail(CHEM_EINVAL, "probe_attempts must be >= 0");
  if (o->method == CHEM_YASS) {
    if (!(o->yass_alpha > 0.0)) return fail(CHEM_EINVAL, "yass_alpha must be positive");
    if (o->linear_solver != CHEM_LINSOLVE_LU && o->linear_solver != CHEM_LINSOLVE_GMRES)
      return fail(CHEM_EINVAL, "unknown linear_solver");
    if (o->krylov_precond != CHEM_PRECOND_NONE && o->krylov_precond != CHEM_PRECOND_JACOBI &&
        o->krylov_precond != CHEM_PRECOND_GAUSS_SEIDEL)
      return fail(CHEM_EINVAL, "unknown krylov_precond");
    if (o->krylov_dim < 0 || o->krylov_max_iter < 1 || !(o->krylov_rtol >= 0.0))
      return fail(CHEM_EINVAL, "krylov_dim >= 0, krylov_max_iter >= 1 and krylov_rtol >= 0 required");
  }
  return CHEM_OK;
}

// the full-system build of a register-resident mechanism (groups 1 to 3: every integrator and the
// adjoints), once; the kernels of group 0 come from the regular build.  Called under M->mu.
chem_err load_full_system(chem_mech* M) {
  if (M->full_loaded) return CHEM_OK;
  std::vector<CodeObject> objs;
  if (chem_err e = build_code_objects(M->m, M->arch, M->cache_dir, objs, true)) return e;
  for (auto& o : objs) {
    hipModule_t md = nullptr;
    HIP_TRY(hipModuleLoadData(&md, o.code.data()));
    M->modules_full.push_back(md);
  }
  for (int k = 0; k < K_COUNT; ++k) {
    const int g = kKernelGroup[k];
    M->fn_full[k] = M->fn[k];
    if (g < 1 || g > 3 || lu_strategy_kernel(k)) continue;
    HIP_TRY(hipModuleGetFunction(&M->fn_full[k], M->modules_full[g - 1], kKernelNames[k]));
  }
  M->full_loaded = true;
  return CHEM_OK;
}

// dynamic LDS of a launch: the Rosenbrock kernels park the upper LU factor of each lane
// (register-resident mechanisms only)
unsigned shmem_for(const chem_mech* M, KernelId k, int block) {
  if (!M->dense || (k != K_ROS2_PERSISTENT && k != K_ROS2_PERSISTENT_REC && k != K_ROS2_STEP)) return 0;
  const int na = solved_size(M);
  return static_cast<unsigned>(na * (na + 1) / 2) * static_cast<unsigned>(block) * sizeof(double);
}

bool shmem_fits(const chem_mech* M, KernelId k, int block) { return shmem_for(M, k, block) <= M->max_shmem; }

// blocks per CU the runtime reports for a kernel at this block size (>= 1)
int occupancy_blocks(const chem_mech* M, KernelId k, int block) {
  int nb = 0;
  if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel_fn(M, k), block, shmem_for(M, k, block)) != hipSuccess ||
      nb < 1)
    nb = 1;
  return nb;
}

// the persistent kernel of a method under the mechanism's LU strategy (strategy 1 only where its
// kernel exists: block form with the factors in LDS; a run that records a tape uses strategy 0,
// the one the adjoint's replays use)
KernelId persistent_kernel_of(const chem_mech* M, int method, bool tape = false) {
  const KernelId k = persistent_kernel(method);
  if (tape || M->lu_strategy[method] != 1) return k;
  if (method == CHEM_ROS2 && M->fn[K_ROS2_PERSISTENT_LUP]) return K_ROS2_PERSISTENT_LUP;
  if (method == CHEM_BE && M->fn[K_BE_PERSISTENT_LUP]) return K_BE_PERSISTENT_LUP;
  return k;
}

void persistent_config(const chem_mech* M, int method, KernelId k, int& block, unsigned& grid) {
  block = M->launch_block[method][CHEM_PERSISTENT] ? M->launch_block[method][CHEM_PERSISTENT] : 64;
  if (M->wave) block = kBlockThreads;
  // the Rosenbrock kernels' LDS grows with the block; 64 fits every register-resident size
  while (block > 64 && !shmem_fits(M, k, block)) block /= 2;
  grid = M->launch_grid[method][CHEM_PERSISTENT]
             ? static_cast<unsigned>(M->launch_grid[method][CHEM_PERSISTENT])
             : static_cast<unsigned>(occupancy_blocks(M, k, block) * M->num_cu);
}

}  // namespace

// ============================================================================ ABI
extern "C" {

void chem_default_options(chem_integrator_opts* o) {
  if (!o) return;
  o->method = CHEM_BE;
  o->energy = CHEM_CONST_P;
  o->form = CHEM_PERSISTENT;
  o->flags = 0;
  o->dt = 1e-7;
  o->n_steps = 0;
  o->max_steps = 100000;
  o->rtol = 1e-6;
  o->atol = 1e-10;
  o->h_min = 1e-20;
  o->newton_max = 10;
  o->halving_max_depth = 8;
  o->newton_rtol = 1e-10;
  o->newton_atol_T = 1e-8;
  o->newton_atol_Y = 1e-14;
  o->probe_attempts = 48;
  o->reserved_ = 0;
  o->yass_alpha = 0.1;
  o->linear_solver = CHEM_LINSOLVE_LU;
  o->krylov_dim = 0;
  o->krylov_rtol = 1e-12;
  o->krylov_max_iter = 100;
  o->krylov_precond = CHEM_PRECOND_JACOBI;
}

const char* chem_error_string(chem_err e) {
  switch (e) {
    case CHEM_OK: return "ok";
    case CHEM_EINVAL: return "invalid argument";
    case CHEM_ENOMEM: return "out of memory";
    case CHEM_EPARSE: return "mechanism parse error";
    case CHEM_EDEVICE: return "HIP device error";
    case CHEM_ECOMPILE: return "kernel compilation failed";
    case CHEM_ECELLS: return "one or more cells failed";
    case CHEM_EUNSUPPORTED: return "unsupported request";
  }
  return "unknown error";
}

const char* chem_last_error_message(void) { return g_last_error.c_str(); }

chem_err chem_precompile(const char* path, const char* cache_dir, char* path_out, size_t cap) {
  chem::Mechanism m;
  chem_err e = parse_file(path, m);
  if (e) return e;
  std::vector<CodeObject> objs;
  e = build_code_objects(m, "gfx950", cache_dir ? cache_dir : default_cache_dir(), objs);
  if (e) return e;
  if (m.n() <= kDenseLimit) {  // the full-system build too (its paths are not reported)
    std::vector<CodeObject> full;
    if ((e = build_code_objects(m, "gfx950", cache_dir ? cache_dir : default_cache_dir(), full, true))) return e;
  }
  if (path_out && cap) {
    std::string paths;
    for (auto& o : objs) paths += (paths.empty() ? "" : ";") + o.path;
    std::strncpy(path_out, paths.c_str(), cap - 1);
    path_out[cap - 1] = '\0';
  }
  return CHEM_OK;
}

chem_err chem_load_mechanism(const char* path, const char* cache_dir, chem_mech** out) {
  if (!out) return fail(CHEM_EINVAL, "null output pointer");
  *out = nullptr;
  std::unique_ptr<chem_mech> M(new chem_mech());
  chem_err e = parse_file(path, M->m);
  if (e) return e;
  HIP_TRY(hipGetDevice(&M->device));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, M->device));
  M->num_cu = prop.multiProcessorCount;
  M->max_shmem = prop.sharedMemPerBlock;
  std::string arch = prop.gcnArchName;
  M->arch = arch.substr(0, arch.find(':'));
  std::vector<CodeObject> objs;
  e = build_code_objects(M->m, M->arch, cache_dir ? cache_dir : default_cache_dir(), objs);
  if (e) return e;
  for (auto& o : objs) {
    hipModule_t md = nullptr;
    HIP_TRY(hipModuleLoadData(&md, o.code.data()));
    M->modules.push_back(md);
  }
  M->dense = M->m.n() <= kDenseLimit;
  M->wave = !M->dense;
  M->wave_api = M->wave && M->m.n() <= kWaveApiLimit;
  M->np = (M->m.n() + 15) / 16 * 16;
  for (int k = 0; k < K_COUNT; ++k) {
    if (M->wave && dense_only(k)) continue;
    hipModule_t md = M->modules[M->modules.size() == 1 ? 0 : kKernelGroup[k]];
    const hipError_t ge = hipModuleGetFunction(&M->fn[k], md, kKernelNames[k]);
    // the block form has no plain-form step kernels (and mechanisms without LDS-resident factors no
    // second LU strategy): those stay null and the entry points that need them refuse the request
    if (ge != hipSuccess && !lu_strategy_kernel(k) &&
        !(M->wave && (k == K_ROS2_STEP || k == K_BE_STEP || k == K_BE_ADJOINT))) {
      HIP_TRY(ge);
    }
    if (ge != hipSuccess) {
      M->fn[k] = nullptr;
      (void)hipGetLastError();  // the expected miss must not stay the thread's last HIP error
    }
  }
  {
    std::vector<bool> act(M->m.ns(), false);
    for (int j = 0; j < M->m.nr(); ++j)
      for (auto& p : M->m.net(j)) act[p.first] = true;
    M->n_active = 1 + static_cast<int>(std::count(act.begin(), act.end(), true));
  }
  M->cache_dir = cache_dir ? cache_dir : default_cache_dir();
  std::vector<double> lnA(std::max(1, M->m.nr()), 0.0);
  for (int j = 0; j < M->m.nr(); ++j) lnA[j] = M->m.reactions[j].k.lnA;
  if ((e = M->lnA_default.ensure(lnA.size() * sizeof(double)))) return e;
  HIP_TRY(hipMemcpy(M->lnA_default.p, lnA.data(), lnA.size() * sizeof(double), hipMemcpyHostToDevice));
  if ((e = M->queue.ensure(sizeof(uint64_t)))) return e;
  if ((e = M->running.ensure(64 * sizeof(unsigned int)))) return e;
  HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&M->running_host), sizeof(unsigned int), hipHostMallocDefault));
  HIP_TRY(hipEventCreateWithFlags(&M->fence, hipEventDisableTiming));
  {
    void* sp = nullptr;
    HIP_TRY(chem_noalloc::scratch_address(M->device, &sp));
    M->scratch = static_cast<unsigned char*>(sp);
  }
  *out = M.release();
  return CHEM_OK;
}

void chem_free_mechanism(chem_mech* mech) { delete mech; }

chem_err chem_mechanism_info(const chem_mech* M, int* ns, int* nr, int* ne, int* n) {
  if (!M) return fail(CHEM_EINVAL, "null mechanism");
  if (ns) *ns = M->m.ns();
  if (nr) *nr = M->m.nr();
  if (ne) *ne = static_cast<int>(M->m.elements.size());
  if (n) *n = M->m.n();
  return CHEM_OK;
}

chem_err chem_molecular_weights(const chem_mech* M, double* W) {
  if (!M || !W) return fail(CHEM_EINVAL, "null argument");
  for (int i = 0; i < M->m.ns(); ++i) W[i] = M->m.species[i].W;
  return CHEM_OK;
}

chem_err chem_default_lnA(const chem_mech* M, double* lnA) {
  if (!M || !lnA) return fail(CHEM_EINVAL, "null argument");
  for (int j = 0; j < M->m.nr(); ++j) lnA[j] = M->m.reactions[j].k.lnA;
  return CHEM_OK;
}

chem_err chem_thermo(const chem_mech* M, int64_t n, int64_t ld, const double* T, double* cp, double* h, double* s,
                     double* g, void* stream) {
  if (!M || !T) return fail(CHEM_EINVAL, "null argument");
  if (chem_err e = check_cells(n, ld)) return e;
  void* args[] = {&n, &ld, &T, &cp, &h, &s, &g};
  return launch(M, K_THERMO, blocks_for(n, 256), 256, static_cast<hipStream_t>(stream), args);
}

chem_err chem_T_from_energy(const chem_mech* M, int64_t n, int64_t ld, const double* C, const double* e,
                            const double* T0, int energy, int n_iter, double* T, void* stream) {
  if (!M || !C || !e || !T0 || !T) return fail(CHEM_EINVAL, "null argument");
  if (chem_err err = check_cells(n, ld)) return err;
  if (!known_energy(energy)) return fail(CHEM_EINVAL, "unknown energy mode");
  if (n_iter < 1) return fail(CHEM_EINVAL, "n_iter must be >= 1");
  void* args[] = {&n, &ld, &C, &e, &T0, &energy, &n_iter, &T};
  return launch(M, K_T_FROM_ENERGY, blocks_for(n, 256), 256, static_cast<hipStream_t>(stream), args);
}

chem_err chem_cfd_source(const chem_mech* M, int64_t n, int64_t ld, const double* y_n, const double* y_np1, double dt,
                         double* R, void* stream) {
  if (!M || !y_n || !y_np1 || !R) return fail(CHEM_EINVAL, "null argument");
  if (chem_err err = check_cells(n, ld)) return err;
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(CHEM_EINVAL, "dt must be positive and finite");
  double inv_dt = 1.0 / dt;
  void* args[] = {&n, &ld, &y_n, &y_np1, &inv_dt, &R};
  return launch(M, K_CFD_SOURCE, blocks_for(n, 256), 256, static_cast<hipStream_t>(stream), args);
}

chem_err chem_source_terms(const chem_mech* M, int64_t n, int64_t ld, const double* y, const double* lnA, int energy,
                           double* dydt, void* stream) {
  if (!M || !y || !dydt) return fail(CHEM_EINVAL, "null argument");
  if (chem_err e = check_cells(M, n, ld)) return e;
  if (!known_energy(energy)) return fail(CHEM_EINVAL, "unknown energy mode");
  const double* la = lnA ? lnA : M->lnA_default.as<double>();
  void* args[] = {&n, &ld, &y, &la, &energy, &dydt};
  if (M->wave && !M->wave_api)  // one cell per workgroup
    return launch(M, K_SOURCE, static_cast<unsigned>(n), kBlockThreads, static_cast<hipStream_t>(stream), args);
  return launch(M, K_SOURCE, blocks_for(n, 256), 256, static_cast<hipStream_t>(stream), args);
}

chem_err chem_jacobian(const chem_mech* M, int64_t n, int64_t ld, const double* y, const double* lnA, int energy,
                       double* jac, void* stream) {
  if (!M || !y || !jac) return fail(CHEM_EINVAL, "null argument");
  if (chem_err e = check_cells(M, n, ld)) return e;
  if (!known_energy(energy)) return fail(CHEM_EINVAL, "unknown energy mode");
  const double* la = lnA ? lnA : M->lnA_default.as<double>();
  void* args[] = {&n, &ld, &y, &la, &energy, &jac};
  if (M->wave) {
    // one wave per cell into a cell-major staging buffer, then a tiled transpose to the SoA
    // layout; cells are processed in chunks so that the staging buffer stays bounded
    const int64_t NN = static_cast<int64_t>(M->m.n()) * M->m.n();
    const int64_t chunk = std::min<int64_t>(n, 32768);
    if (n == 0) return CHEM_OK;
    chem_mech* Mm = const_cast<chem_mech*>(M);
    std::lock_guard<std::mutex> lock(Mm->mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    StreamFence fence(Mm, s);
    if (chem_err e = fence.begin()) return e;
    if (chem_err e = Mm->jstage.ensure(sizeof(double) * static_cast<size_t>(chunk * NN))) return e;
    double* stage = Mm->jstage.as<double>();
    for (int64_t c0 = 0; c0 < n; c0 += chunk) {
      int64_t nc = std::min(chunk, n - c0);
      {
        void* a[] = {&nc, &ld, &y, &la, &energy, &stage, &c0};
        if (chem_err e = launch(M, K_JACOBIAN, static_cast<unsigned>(nc), M->wave_api ? 64 : kBlockThreads, s, a))
          return e;
      }
      {
        void* a[] = {&nc, &ld, &stage, &c0, &jac};
        if (chem_err e = launch2d(M, K_JAC_TRANSPOSE, static_cast<unsigned>((NN + 63) / 64),
                                  static_cast<unsigned>((nc + 63) / 64), 256, s, a))
          return e;
      }
    }
    return CHEM_OK;
  }
  return launch(M, K_JACOBIAN, blocks_for(n, 256), 256, static_cast<hipStream_t>(stream), args);
}

chem_err chem_state_from_TPY(const chem_mech* M, int64_t n, int64_t ld, const double* T, const double* p,
                             const double* Y, double* y, void* stream) {
  if (!M || !T || !p || !Y || !y) return fail(CHEM_EINVAL, "null argument");
  if (chem_err e = check_cells(n, ld)) return e;
  void* args[] = {&n, &ld, &T, &p, &Y, &y};
  return launch(M, K_TPY, blocks_for(n, 256), 256, static_cast<hipStream_t>(stream), args);
}

chem_err chem_mass_fractions(const chem_mech* M, int64_t n, int64_t ld, const double* y, double* Y, void* stream) {
  if (!M || !y || !Y) return fail(CHEM_EINVAL, "null argument");
  if (chem_err e = check_cells(n, ld)) return e;
  void* args[] = {&n, &ld, &y, &Y};
  return launch(M, K_MASSFRAC, blocks_for(n, 256), 256, static_cast<hipStream_t>(stream), args);
}

chem_err chem_state_from_TPY_vjp(const chem_mech* M, int64_t n, int64_t ld, const double* T, const double* p,
                                 const double* Y, const double* dLdy, double* dT, double* dY, void* stream) {
  if (!M || !T || !p || !Y || !dLdy || !dT || !dY) return fail(CHEM_EINVAL, "null argument");
  if (chem_err e = check_cells(n, ld)) return e;
  void* args[] = {&n, &ld, &T, &p, &Y, &dLdy, &dT, &dY};
  return launch(M, K_TPY_VJP, blocks_for(n, 256), 256, static_cast<hipStream_t>(stream), args);
}

chem_err chem_mass_fractions_vjp(const chem_mech* M, int64_t n, int64_t ld, const double* y, const double* dY,
                                 const double* dT, double* out, void* stream) {
  if (!M || !y || !dY || !out) return fail(CHEM_EINVAL, "null argument");
  if (chem_err e = check_cells(n, ld)) return e;
  void* args[] = {&n, &ld, &y, &dY, &dT, &out};
  return launch(M, K_MASSFRAC_VJP, blocks_for(n, 256), 256, static_cast<hipStream_t>(stream), args);
}

chem_err chem_tape_create(const chem_mech* M, int64_t n_cells, int ckpt_every, chem_tape** out) {
  if (!M || !out) return fail(CHEM_EINVAL, "null argument");
  if (n_cells < 0 || ckpt_every < 1) return fail(CHEM_EINVAL, "n_cells >= 0 and checkpoint_every >= 1 required");
  chem_tape* t = new chem_tape();
  t->mech = M;
  t->n_cells = n_cells;
  t->ckpt_every = ckpt_every;
  *out = t;
  return CHEM_OK;
}

chem_err chem_tape_create_ros2(const chem_mech* M, int64_t n_cells, int max_steps, int ckpt_every, chem_tape** out) {
  if (!M || !out) return fail(CHEM_EINVAL, "null argument");
  if (n_cells < 0 || max_steps < 1 || ckpt_every < 1)
    return fail(CHEM_EINVAL, "n_cells >= 0, max_steps >= 1 and checkpoint_every >= 1 required");
  if (M->wave) return fail(CHEM_EUNSUPPORTED, "the Rosenbrock adjoint is implemented for n <= 24");
  chem_tape* t = new chem_tape();
  t->mech = M;
  t->method = CHEM_ROS2;
  t->n_cells = n_cells;
  t->max_steps = max_steps;
  t->ckpt_every = ckpt_every;
  *out = t;
  return CHEM_OK;
}

void chem_tape_free(chem_tape* t) { delete t; }

static chem_err fill_u64(chem_mech* M, uint64_t* p, int n, uint64_t v, hipStream_t s) {
  void* args[] = {&p, &n, &v};
  return launch(M, K_FILL_U64, blocks_for(n, 64), 64, s, args);
}

}  // extern "C"

namespace {

// Device workspaces supplied by the caller of integrate_impl instead of the mechanism's own
// buffers (the allocation-free entry point).  Sized for n <= max_cells and, when counters is
// used, ld <= max_cells.
struct FixedWorkspace {
  uint64_t* queue;
  unsigned int* sched;
  double* wst;
  int* order;
  int* counters;
  int64_t max_cells;
};

chem_err integrate_impl(chem_mech* M, int64_t n, int64_t ld, double* y, const double* lnA,
                        const chem_integrator_opts* opts, chem_tape* tape, int32_t* status, int32_t* counters,
                        void* stream, const FixedWorkspace* fw);

}  // namespace

extern "C" {

chem_err chem_integrate(const chem_mech* Mc, int64_t n, int64_t ld, double* y, const double* lnA,
                        const chem_integrator_opts* opts, chem_tape* tape, int32_t* status, int32_t* counters,
                        void* stream) {
  return integrate_impl(const_cast<chem_mech*>(Mc), n, ld, y, lnA, opts, tape, status, counters, stream, nullptr);
}

chem_err chem_integrate_noalloc(const chem_mech* Mc, int64_t n, int64_t ld, double* y, const double* lnA,
                                const chem_integrator_opts* opts, int32_t* status, int32_t* counters, void* stream) {
  chem_mech* M = const_cast<chem_mech*>(Mc);
  if (!M || !opts) return fail(CHEM_EINVAL, "null argument");
  if (opts->form != CHEM_PERSISTENT) return fail(CHEM_EINVAL, "chem_integrate_noalloc runs the persistent form only");
  if (opts->flags & CHEM_FLAG_CHECK_CELLS)
    return fail(CHEM_EINVAL, "CHEM_FLAG_CHECK_CELLS is not available in chem_integrate_noalloc");
  if (n > chem_noalloc::kMaxCells)
    return fail(CHEM_EINVAL, "chem_integrate_noalloc takes at most " + std::to_string(chem_noalloc::kMaxCells) +
                                 " cells per call (got " + std::to_string(n) + ")");
  if (!counters && ld > chem_noalloc::kMaxCells)
    return fail(CHEM_EINVAL, "chem_integrate_noalloc without a counters array needs ld <= " +
                                 std::to_string(chem_noalloc::kMaxCells));
  if (!M->scratch) return fail(CHEM_EDEVICE, "the scratch array of this device is not resolved");
  FixedWorkspace fw{reinterpret_cast<uint64_t*>(M->scratch + chem_noalloc::kQueueOff),
                    reinterpret_cast<unsigned int*>(M->scratch + chem_noalloc::kSchedOff),
                    reinterpret_cast<double*>(M->scratch + chem_noalloc::kWstOff),
                    reinterpret_cast<int*>(M->scratch + chem_noalloc::kOrderOff),
                    reinterpret_cast<int*>(M->scratch + chem_noalloc::kCountersOff), chem_noalloc::kMaxCells};
  return integrate_impl(M, n, ld, y, lnA, opts, nullptr, status, counters, stream, &fw);
}

}  // extern "C"

namespace {

chem_err integrate_impl(chem_mech* M, int64_t n, int64_t ld, double* y, const double* lnA,
                        const chem_integrator_opts* opts, chem_tape* tape, int32_t* status, int32_t* counters,
                        void* stream, const FixedWorkspace* fw) {
  if (!M || !y || !status) return fail(CHEM_EINVAL, "null argument");
  if (chem_err e = check_cells(M, n, ld)) return e;
  if (chem_err e = validate_opts(opts)) return e;
  if (chem_err e = check_reactor(M, opts, tape != nullptr)) return e;
  if (M->wave) {
    // the block form (n > 24): backward Euler and Rosenbrock, persistent form; adjoint tapes for
    // backward Euler only
    if (opts->method != CHEM_BE && opts->method != CHEM_ROS2)
      return fail(CHEM_EUNSUPPORTED, std::string(method_name(opts->method)) + " is implemented for n <= 24");
    if (opts->form != CHEM_PERSISTENT)
      return fail(CHEM_EUNSUPPORTED, "mechanisms with n > 24 integrate in the persistent form");
    if (tape && (opts->method != CHEM_BE || !M->fn[K_BE_ADJOINT]))
      return fail(CHEM_EUNSUPPORTED, "mechanisms with n > 24 record adjoint tapes for backward Euler only");
    if (fw && M->np > 64)
      return fail(CHEM_EUNSUPPORTED, "chem_integrate_noalloc covers mechanisms with n <= 64");
  }
  if (persistent_only(opts->method)) {
    if (opts->form != CHEM_PERSISTENT)
      return fail(CHEM_EUNSUPPORTED, std::string(method_name(opts->method)) + " runs in the persistent form only");
    if (tape) return fail(CHEM_EUNSUPPORTED, std::string("no adjoint tape for ") + method_name(opts->method));
  }
  if (tape) {
    if (tape->mech != M) return fail(CHEM_EINVAL, "tape belongs to another mechanism");
    if (tape->method != opts->method) return fail(CHEM_EINVAL, "tape was created for another method");
    // the backward-Euler tape stores each step's substep count (at most 2^depth) as 16 bits
    if (tape->method == CHEM_BE && opts->halving_max_depth > 15)
      return fail(CHEM_EINVAL, "halving_max_depth <= 15 is required when recording a backward-Euler tape");
    if (tape->n_cells < n) return fail(CHEM_EINVAL, "tape was created for fewer cells");
    if (tape->method == CHEM_ROS2 && opts->form != CHEM_PERSISTENT)
      return fail(CHEM_EUNSUPPORTED, "Rosenbrock recording runs in the persistent form");
  }
  if (n == 0) return CHEM_OK;
  std::lock_guard<std::mutex> lock(M->mu);
  // the reactor mode of a register-resident mechanism runs the full-system build (compiled or
  // fetched from the cache and loaded on first use; the allocation-free entry point only uses it
  // once loaded)
  const bool full = opts->energy == CHEM_CONST_P_REACTOR && M->dense;
  if (full && !M->full_loaded) {
    if (fw)
      return fail(CHEM_EUNSUPPORTED, "the reactor mode of this mechanism needs its full-system build, which "
                  "chem_integrate_noalloc does not load (run chem_integrate once in that mode first)");
    if (chem_err e = load_full_system(M)) return e;
  }
  FullSystemScope scope(full);
  hipStream_t s = static_cast<hipStream_t>(stream);
  StreamFence fence(M, s);
  if (chem_err e = fence.begin()) return e;
  const double* la = lnA ? lnA : M->lnA_default.as<double>();
  const int NY = M->m.n();
  DevChemOpts o = to_dev(*opts, tape ? tape->ckpt_every : 1);
  chem_err e;
  int* cnt = counters;
  if (!cnt && fw) {
    cnt = fw->counters;
  } else if (!cnt) {
    if ((e = M->counters_internal.ensure(sizeof(int) * 3 * static_cast<size_t>(ld)))) return e;
    cnt = M->counters_internal.as<int>();
  }
  double* ckpt = nullptr;
  unsigned short* nsub = nullptr;
  double* hs = nullptr;
  int* nacc = nullptr;
  int cap = 0;
  if (tape && tape->method == CHEM_ROS2) {
    // step sizes of up to max_steps accepted steps, states every ckpt_every steps
    cap = tape->max_steps;
    const int slots = cap / o.ckpt_every + 1;
    if ((e = tape->ckpt.ensure(sizeof(double) * static_cast<size_t>(slots) * NY * ld))) return e;
    if ((e = tape->hs.ensure(sizeof(double) * static_cast<size_t>(cap) * ld))) return e;
    if ((e = tape->nacc.ensure(sizeof(int) * static_cast<size_t>(ld)))) return e;
    if ((e = tape->status.ensure(sizeof(int) * static_cast<size_t>(ld)))) return e;
    ckpt = tape->ckpt.as<double>();
    hs = tape->hs.as<double>();
    nacc = tape->nacc.as<int>();
    // initial states = checkpoint 0 (same [n][ld] layout); the adjoint rebuilds the others
    HIP_TRY(hipMemcpyAsync(ckpt, y, sizeof(double) * static_cast<size_t>(NY) * ld, hipMemcpyDeviceToDevice, s));
    tape->ld = ld;
    tape->n_cells = n;
    tape->opts = o;
    tape->recorded = false;
  } else if (tape) {
    const int slots = o.n_steps / o.ckpt_every + 1;
    if ((e = tape->ckpt.ensure(sizeof(double) * static_cast<size_t>(slots) * NY * ld))) return e;
    if ((e = tape->nsub.ensure(sizeof(unsigned short) * static_cast<size_t>(o.n_steps) * ld))) return e;
    if ((e = tape->status.ensure(sizeof(int) * static_cast<size_t>(ld)))) return e;
    ckpt = tape->ckpt.as<double>();
    nsub = tape->nsub.as<unsigned short>();
    tape->ld = ld;
    tape->n_cells = n;
    tape->opts = o;
    tape->recorded = false;
  }
  const int method = opts->method;
  if (opts->form == CHEM_PERSISTENT) {
    const KernelId k = (method == CHEM_ROS2 && hs) ? K_ROS2_PERSISTENT_REC : persistent_kernel_of(M, method, tape);
    int block;
    unsigned grid;
    persistent_config(M, method, k, block, grid);
    int64_t slots = static_cast<int64_t>(grid) * block;
    double* ws = nullptr;
    if (M->wave && M->np > 64) {
      // the block form's matrix stores: one padded np x np matrix per workgroup of the grid
      if ((e = M->ws.ensure(sizeof(double) * static_cast<size_t>(M->np) * M->np * grid))) return e;
      ws = M->ws.as<double>();
    }
    uint64_t* q = fw ? fw->queue : M->queue.as<uint64_t>();
    if ((e = fill_u64(M, q, 1, 0, s))) return e;
    if (method == CHEM_YASS) {
      DevYassOpts yo = yass_to_dev(*opts);
      void* args[] = {&n, &ld, &y, &la, &o, &yo, &status, &cnt, &q};
      if ((e = launch(M, k, grid, block, s, args))) return e;
    } else if (persistent_only(method)) {
      void* args[] = {&n, &ld, &y, &la, &o, &status, &cnt, &q};
      if ((e = launch(M, k, grid, block, s, args))) return e;
    } else if (method == CHEM_ROS2) {
      const unsigned shm = shmem_for(M, k, block);
      int budget = opts->probe_attempts;
      if (n >= (int64_t(1) << 31)) budget = 0;
      double* wst = nullptr;
      int* order = nullptr;
      unsigned int* sched = nullptr;
      if (budget > 0) {
        // probe launch, bins of the parked cells, resume launch in that order (no host sync)
        if (fw) {
          wst = fw->wst;
          order = fw->order;
          sched = fw->sched;
        } else {
          if ((e = M->wst.ensure(sizeof(double) * 4 * static_cast<size_t>(n)))) return e;
          if ((e = M->order.ensure(sizeof(int) * static_cast<size_t>(n)))) return e;
          // [0] parked count, [1, 1 + bins) bin counts, [1 + bins, 1 + 2 bins) bin offsets, 1 pad word
          if ((e = M->sched.ensure(sizeof(unsigned int) * (2 + 2 * kSchedBins)))) return e;
          wst = M->wst.as<double>();
          order = M->order.as<int>();
          sched = M->sched.as<unsigned int>();
        }
        if ((e = fill_u64(M, reinterpret_cast<uint64_t*>(sched), (2 + 2 * kSchedBins) / 2, 0, s))) return e;
      }
      const int* no_order = nullptr;
      void* args[] = {&n,   &ld,       &y,     &la, &o,    &status, &cnt, &q, &ws, &slots, &budget,
                      &wst, &no_order, &sched, &hs, &nacc, &cap};
      if ((e = launch(M, k, grid, block, s, args, shm))) return e;
      if (budget > 0) {
        {
          void* a2[] = {&sched};
          if ((e = launch(M, K_SCHED_SCAN, 1, kSchedBins, s, a2))) return e;
        }
        {
          void* a3[] = {&n, &status, &wst, &sched, &order};
          if ((e = launch(M, K_SCHED_SCATTER, blocks_for(n, 256), 256, s, a3))) return e;
        }
        if ((e = fill_u64(M, q, 1, 0, s))) return e;
        int zero = 0;
        void* a4[] = {&n, &ld, &y, &la, &o, &status, &cnt, &q, &ws, &slots, &zero, &wst, &order, &sched,
                      &hs, &nacc, &cap};
        if ((e = launch(M, k, grid, block, s, a4, shm))) return e;
      }
    } else {
      void* args[] = {&n, &ld, &y, &la, &o, &status, &cnt, &q, &ws, &slots, &ckpt, &nsub};
      if ((e = launch(M, k, grid, block, s, args))) return e;
    }
  } else {
    int block = M->wave ? 64 : (M->launch_block[method][CHEM_PLAIN] ? M->launch_block[method][CHEM_PLAIN] : 64);
    // the Rosenbrock step parks U in LDS, which grows with the solved system (the full-system build
    // of the reactor mode solves more components than the launch shape may have been set for)
    while (method == CHEM_ROS2 && block > 64 && !shmem_fits(M, K_ROS2_STEP, block)) block /= 2;
    const unsigned grid = M->wave ? static_cast<unsigned>(n) : blocks_for(n, block);
    int64_t slots = n;
    double* ws = nullptr;
    if (!M->dense && !M->wave) {
      if ((e = M->ws.ensure(sizeof(double) * static_cast<size_t>(NY) * NY * slots))) return e;
      ws = M->ws.as<double>();
    }
    if (method == CHEM_ROS2) {
      if ((e = M->wst.ensure(sizeof(double) * 4 * static_cast<size_t>(n)))) return e;
      double* wst = M->wst.as<double>();
      {
        void* args[] = {&n, &ld, &y, &status, &cnt, &wst};
        if ((e = launch(M, K_ROS2_INIT, blocks_for(n, 256), 256, s, args))) return e;
      }
      unsigned int* run = M->running.as<unsigned int>();
      const int batch = 16;
      int64_t launched = 0;
      while (launched <= opts->max_steps) {
        if ((e = fill_u64(M, reinterpret_cast<uint64_t*>(run), 32, 0, s))) return e;
        for (int b = 0; b < batch; ++b) {
          unsigned int* slot = run + b;
          void* args[] = {&n, &ld, &y, &la, &o, &status, &cnt, &wst, &slot, &ws, &slots};
          if ((e = launch(M, K_ROS2_STEP, grid, block, s, args, shmem_for(M, K_ROS2_STEP, block)))) return e;
        }
        launched += batch;
        HIP_TRY(hipMemcpyAsync(M->running_host, run + batch - 1, sizeof(unsigned int), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (*M->running_host == 0) break;
      }
    } else {
      {
        void* args[] = {&n, &ld, &y, &status, &cnt, &ckpt};
        if ((e = launch(M, K_BE_INIT, blocks_for(n, 256), 256, s, args))) return e;
      }
      for (int st = 0; st < o.n_steps; ++st) {
        void* args[] = {&n, &ld, &y, &la, &o, &status, &cnt, &ws, &slots, &ckpt, &nsub};
        if ((e = launch(M, K_BE_STEP, grid, block, s, args))) return e;
      }
    }
  }
  if (tape) {
    HIP_TRY(hipMemcpyAsync(tape->status.p, status, sizeof(int) * static_cast<size_t>(n), hipMemcpyDeviceToDevice, s));
    tape->recorded = true;
  }
  if (opts->flags & CHEM_FLAG_CHECK_CELLS) {
    std::vector<int> h(static_cast<size_t>(n));
    HIP_TRY(hipMemcpyAsync(h.data(), status, sizeof(int) * h.size(), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int v : h)
      if (v != CHEM_CELL_OK) return fail(CHEM_ECELLS, "at least one cell did not finish with status OK");
  }
  return CHEM_OK;
}

}  // namespace

extern "C" {

// Reverse sweep of a Rosenbrock tape: one lane per cell (static grid-stride mapping), segment
// states in M->seg, per-block ln A partial sums reduced in block order.
static chem_err ros2_adjoint(chem_mech* M, chem_tape* tape, const double* la, const double* dLdyN, double* dLdy0,
                             double* dLdlnA, hipStream_t s) {
  int64_t n = tape->n_cells, ld = tape->ld;
  const int NY = M->m.n(), NR = std::max(1, M->m.nr());
  const int block = 256;
  const unsigned cap = static_cast<unsigned>(occupancy_blocks(M, K_ROS2_ADJOINT, block) * M->num_cu);
  const unsigned grid = std::max(1u, std::min(blocks_for(n, block), cap));
  int64_t total = static_cast<int64_t>(grid) * block;
  chem_err e;
  const int K = tape->opts.ckpt_every;
  // per-step records of one segment: state, LU factors and pivots, two stages (SEG_W values)
  const size_t seg_w = 4 * static_cast<size_t>(NY) + static_cast<size_t>(NY) * NY;
  if ((e = M->seg.ensure(sizeof(double) * static_cast<size_t>(K) * seg_w * total))) return e;
  if ((e = M->gpart.ensure(sizeof(double) * static_cast<size_t>(grid) * NR))) return e;
  DevChemOpts o = tape->opts;
  const int* st = tape->status.as<int>();
  const int* na = tape->nacc.as<int>();
  const double* hs = tape->hs.as<double>();
  double* ck = tape->ckpt.as<double>();
  double* seg = M->seg.as<double>();
  double* gp = M->gpart.as<double>();
  {
    void* args[] = {&n, &ld, &la, &o, &st, &na, &hs, &ck, &dLdyN, &dLdy0, &gp, &seg, &total};
    if ((e = launch(M, K_ROS2_ADJOINT, grid, block, s, args))) return e;
  }
  int nb = static_cast<int>(grid);
  void* args[] = {&nb, &gp, &dLdlnA};
  return launch(M, K_REDUCE_BLOCKS, blocks_for(NR, 64), 64, s, args);
}

chem_err chem_integrate_adjoint(const chem_mech* Mc, chem_tape* tape, const double* lnA, const double* dLdyN,
                                double* dLdy0, double* dLdlnA, void* stream) {
  chem_mech* M = const_cast<chem_mech*>(Mc);
  if (!M || !tape || !dLdyN || !dLdy0 || !dLdlnA) return fail(CHEM_EINVAL, "null argument");
  if (tape->mech != M) return fail(CHEM_EINVAL, "tape belongs to another mechanism");
  if (M->wave && (tape->method != CHEM_BE || !M->fn[K_BE_ADJOINT]))
    return fail(CHEM_EUNSUPPORTED, "mechanisms with n > 24 have the backward-Euler adjoint only");
  if (!tape->recorded) return fail(CHEM_EINVAL, "tape holds no recorded forward run");
  std::lock_guard<std::mutex> lock(M->mu);
  // a tape recorded in the reactor mode of a register-resident mechanism is swept by the adjoint of
  // the full-system build (its replays solve for every species)
  const bool full = tape->opts.energy == CHEM_CONST_P_REACTOR && M->dense;
  if (full)
    if (chem_err e = load_full_system(M)) return e;
  FullSystemScope scope(full);
  hipStream_t s = static_cast<hipStream_t>(stream);
  StreamFence fence(M, s);
  if (chem_err e = fence.begin()) return e;
  int64_t n = tape->n_cells, ld = tape->ld;
  const double* la = lnA ? lnA : M->lnA_default.as<double>();
  const int NY = M->m.n(), NR = std::max(1, M->m.nr());
  if (tape->method == CHEM_ROS2) return ros2_adjoint(M, tape, la, dLdyN, dLdy0, dLdlnA, s);
  const int block = 256;
  const unsigned cap = static_cast<unsigned>(occupancy_blocks(M, K_BE_ADJOINT, block) * M->num_cu);
  const unsigned grid = std::max(1u, std::min(M->wave ? static_cast<unsigned>(std::min<int64_t>(n, 1 << 30))
                                                      : blocks_for(n, block), cap));
  // state slots of the segment recompute: one per lane, or one per workgroup in the block form
  int64_t total = M->wave ? static_cast<int64_t>(grid) : static_cast<int64_t>(grid) * block;
  chem_err e;
  const int K = tape->opts.ckpt_every;
  if ((e = M->seg.ensure(sizeof(double) * static_cast<size_t>(K) * NY * total))) return e;
  if ((e = M->gpart.ensure(sizeof(double) * static_cast<size_t>(grid) * NR))) return e;
  double* ws = nullptr;
  double* gws = nullptr;
  if (!M->dense && !M->wave) {
    if ((e = M->ws.ensure(sizeof(double) * static_cast<size_t>(NY) * NY * total))) return e;
    if ((e = M->gws.ensure(sizeof(double) * static_cast<size_t>(NR) * total))) return e;
    ws = M->ws.as<double>();
    gws = M->gws.as<double>();
  } else if (M->wave && M->np > 64) {
    // block form with the factors in device memory: one padded matrix per workgroup
    if ((e = M->ws.ensure(sizeof(double) * static_cast<size_t>(M->np) * M->np * grid))) return e;
    ws = M->ws.as<double>();
  }
  DevChemOpts o = tape->opts;
  const int* st = tape->status.as<int>();
  const double* ck = tape->ckpt.as<double>();
  const unsigned short* ns = tape->nsub.as<unsigned short>();
  double* seg = M->seg.as<double>();
  double* gp = M->gpart.as<double>();
  {
    void* args[] = {&n, &ld, &la, &o, &st, &ck, &ns, &dLdyN, &dLdy0, &gp, &seg, &total, &ws, &total, &gws};
    if ((e = launch(M, K_BE_ADJOINT, grid, block, s, args))) return e;
  }
  int nb = static_cast<int>(grid);
  void* args[] = {&nb, &gp, &dLdlnA};
  return launch(M, K_REDUCE_BLOCKS, blocks_for(NR, 64), 64, s, args);
}

chem_err chem_set_launch(chem_mech* M, int method, int form, int block, int grid) {
  if (!M) return fail(CHEM_EINVAL, "null mechanism");
  if (!known_method(method) ||
      (form != CHEM_PERSISTENT && form != CHEM_PLAIN))
    return fail(CHEM_EINVAL, "unknown method or form");
  if (block != 0 && (block < 64 || block > kMaxBlock || block % 64)) return fail(CHEM_EINVAL, "block must be 64..256, a multiple of 64");
  if (grid < 0) return fail(CHEM_EINVAL, "grid must be >= 0");
  if (block != 0 && method == CHEM_ROS2 && !M->wave) {
    const KernelId k = form == CHEM_PERSISTENT ? K_ROS2_PERSISTENT : K_ROS2_STEP;
    if (!shmem_fits(M, k, block))
      return fail(CHEM_EINVAL, "block " + std::to_string(block) + " needs " + std::to_string(shmem_for(M, k, block)) +
                                   " B of LDS for the Rosenbrock kernel; the device allows " +
                                   std::to_string(M->max_shmem));
  }
  M->launch_block[method][form] = M->wave && block != 0 ? kBlockThreads : block;
  M->launch_grid[method][form] = grid;
  return CHEM_OK;
}

chem_err chem_get_launch(const chem_mech* M, int method, int form, int* block, int* grid) {
  if (!M || !block || !grid) return fail(CHEM_EINVAL, "null argument");
  if (!known_method(method) ||
      (form != CHEM_PERSISTENT && form != CHEM_PLAIN))
    return fail(CHEM_EINVAL, "unknown method or form");
  if (form == CHEM_PERSISTENT) {
    int b;
    unsigned g;
    persistent_config(M, method, persistent_kernel_of(M, method), b, g);
    *block = b;
    *grid = static_cast<int>(g);
  } else {
    *block = M->wave ? kBlockThreads : (M->launch_block[method][form] ? M->launch_block[method][form] : 64);
    *grid = 0;
  }
  return CHEM_OK;
}

chem_err chem_set_lu_strategy(chem_mech* M, int method, int strategy) {
  if (!M) return fail(CHEM_EINVAL, "null mechanism");
  if (!known_method(method)) return fail(CHEM_EINVAL, "unknown method");
  if (strategy != 0 && strategy != 1) return fail(CHEM_EINVAL, "LU strategy must be 0 or 1");
  if (strategy == 1) {
    const KernelId k = method == CHEM_ROS2 ? K_ROS2_PERSISTENT_LUP : (method == CHEM_BE ? K_BE_PERSISTENT_LUP : K_COUNT);
    if (k == K_COUNT || !M->fn[k])
      return fail(CHEM_EUNSUPPORTED, "LU strategy 1 exists for backward Euler and Rosenbrock of mechanisms with "
                                     "24 < n <= 64 (block form, factors in LDS)");
  }
  M->lu_strategy[method] = strategy;
  return CHEM_OK;
}

chem_err chem_get_lu_strategy(const chem_mech* M, int method, int* strategy) {
  if (!M || !strategy) return fail(CHEM_EINVAL, "null argument");
  if (!known_method(method)) return fail(CHEM_EINVAL, "unknown method");
  *strategy = M->lu_strategy[method];
  return CHEM_OK;
}

chem_err chem_autotune(chem_mech* M, int64_t n, int64_t ld, const double* y, const double* lnA,
                       const chem_integrator_opts* opts, void* stream) {
  if (!M || !y) return fail(CHEM_EINVAL, "null argument");
  if (chem_err e = check_cells(M, n, ld)) return e;
  if (chem_err e = validate_opts(opts)) return e;
  if (opts->form != CHEM_PERSISTENT) return fail(CHEM_EUNSUPPORTED, "autotuning covers the persistent form");
  if (chem_err e = check_reactor(M, opts, false)) return e;
  if (M->wave && opts->method != CHEM_BE && opts->method != CHEM_ROS2)
    return fail(CHEM_EUNSUPPORTED, std::string(method_name(opts->method)) + " is implemented for n <= 24");
  if (n == 0) return CHEM_OK;
  const bool full = opts->energy == CHEM_CONST_P_REACTOR && M->dense;
  if (full) {
    std::lock_guard<std::mutex> lock(M->mu);
    if (chem_err e = load_full_system(M)) return e;
  }
  FullSystemScope scope(full);   // the occupancy queries below see the build the trials run
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int NY = M->m.n();
  DevBuf ycopy, st;
  chem_err e;
  if ((e = ycopy.ensure(sizeof(double) * NY * static_cast<size_t>(ld)))) return e;
  if ((e = st.ensure(sizeof(int) * static_cast<size_t>(ld)))) return e;
  hipEvent_t a, b;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  float best = 1e30f;
  int best_block = 64, best_grid = 0, best_lus = 0;
  const int method = opts->method;
  const int prev_block = M->launch_block[method][CHEM_PERSISTENT], prev_grid = M->launch_grid[method][CHEM_PERSISTENT];
  const int prev_lus = M->lu_strategy[method];
  // LU strategies to try: 1 only where its kernels exist
  std::vector<int> strategies = {0};
  if ((method == CHEM_ROS2 && M->fn[K_ROS2_PERSISTENT_LUP]) || (method == CHEM_BE && M->fn[K_BE_PERSISTENT_LUP]))
    strategies.push_back(1);
  // one timed trial of a launch shape on a copy of the cells
  auto trial = [&](int block, int grid, float& ms) -> chem_err {
    if (chem_err err = chem_set_launch(M, method, CHEM_PERSISTENT, block, grid)) return err;
    HIP_TRY(hipMemcpyAsync(ycopy.p, y, sizeof(double) * NY * static_cast<size_t>(ld), hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipEventRecord(a, s));
    chem_err err = chem_integrate(M, n, ld, ycopy.as<double>(), lnA, opts, nullptr, st.as<int>(), nullptr, stream);
    HIP_TRY(hipEventRecord(b, s));
    HIP_TRY(hipEventSynchronize(b));
    if (err) return err;
    HIP_TRY(hipEventElapsedTime(&ms, a, b));
    return CHEM_OK;
  };
  e = CHEM_OK;
  for (int lus : strategies) {
    M->lu_strategy[method] = lus;
    const KernelId k = persistent_kernel_of(M, method);
    for (int block : {64, 128, 256}) {
      if (M->wave && block != kBlockThreads) continue;  // one cell per 256-thread workgroup
      if (!shmem_fits(M, k, block)) continue;  // the Rosenbrock kernels' LDS grows with the block
      const int occ = occupancy_blocks(M, k, block);
      for (int mult : {1, 2}) {
        const int grid = occ * M->num_cu * mult;
        float ms = 0.f;
        if ((e = trial(block, grid, ms))) break;
        if (ms < best) {
          best = ms;
          best_block = block;
          best_grid = grid;
          best_lus = lus;
        }
      }
      if (e) break;
    }
    if (e) break;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  if (e) {
    // a failed trial leaves the configuration the mechanism had before
    M->launch_block[method][CHEM_PERSISTENT] = prev_block;
    M->launch_grid[method][CHEM_PERSISTENT] = prev_grid;
    M->lu_strategy[method] = prev_lus;
    return e;
  }
  M->lu_strategy[method] = best_lus;
  return chem_set_launch(M, method, CHEM_PERSISTENT, best_block, best_grid);
}

}  // extern "C"
