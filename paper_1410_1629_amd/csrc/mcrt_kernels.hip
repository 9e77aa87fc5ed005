// mcrt_kernels.hip -- gfx950 kernels of the photon-package life cycle and the
// C ABI that launches them (declared in include/mcrt.h).
//
// Method: Camps & Baes (arXiv:1410.1629), Sect. 1 (photon packages; peel-off
// at emission and scattering; continuous absorption; forced scattering),
// Sect. 2.1-2.3 (multiple anisotropic scattering; cells of constant
// properties; geometries; frames; optical properties).
//
// Execution model.  One package per lane (mcrt_lane.hpp holds the per-lane
// state machine and the walk step).  The life-cycle kernel is persistent:
// every state that needs a walk through the grid sets up a ray, and all rays,
// whatever they are for (peel-off, pass-1 path, pass-2 locate, adjoint
// deposit), advance together in one loop, one cell crossing per iteration,
// so the lanes of a wavefront stay in the walk whatever event their packages
// are at.  A wavefront leaves the walk to run events only once `batch` of
// its lanes are waiting (or none is walking).  Lanes that finish a package
// take the next from a global counter, one atomic per wavefront.  The
// adjoint kernel runs the same machine twice per package, so paths are
// recomputed from the random numbers, never stored.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "mcrt.h"
#include "mcrt_device.hpp"
#include "mcrt_attached.hpp"
#include "mcrt_host.hpp"
#include "mcrt_lane.hpp"

namespace mcrt {

constexpr int kBlock = 256;

// ---------------------------------------------------------------------------
// Wave-level helpers (wave64).

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ void atomic_add_f64(double* p, double v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ unsigned long long shfl_u64(unsigned long long v, int src) {
  const unsigned lo = __shfl((unsigned)v, src), hi = __shfl((unsigned)(v >> 32), src);
  return ((unsigned long long)hi << 32) | lo;
}

// One work item for every calling lane.  Each wavefront keeps a reservoir
// [res[0], res[1]) of items in LDS, touched only by its leading calling lane,
// and refills it with one global atomic per `chunk` items, so the single
// global counter sees few, large requests.
__device__ __forceinline__ unsigned long long wave_fetch(unsigned long long* counter, unsigned long long* res,
                                                         unsigned chunk) {
  const unsigned long long m = __ballot(1);
  const int lane = __lane_id();
  const int leader = __ffsll((long long)m) - 1;
  const unsigned rank = __popcll(m & ((1ull << lane) - 1ull));
  const unsigned cnt = __popcll(m);
  unsigned long long a = 0, avail = 0, nb = 0;
  if (lane == leader) {
    a = res[0];
    avail = res[1] - a;
    if (avail >= cnt) {
      res[0] = a + cnt;
    } else {
      const unsigned long long need = cnt - avail, take = need > chunk ? need : chunk;
      nb = atomicAdd(counter, take);
      res[0] = nb + need;
      res[1] = nb + take;
    }
  }
  a = shfl_u64(a, leader);
  avail = shfl_u64(avail, leader);
  nb = shfl_u64(nb, leader);
  return rank < avail ? a + rank : nb + (rank - avail);
}

constexpr int kWavesPerBlock = kBlock / 64;

// Counter block of a life-cycle call (u64 words): [0] next work item,
// [8..10] FP64 luminosity stats, [16..22] crossing and event counts,
// [24] next peel-job slot, [25] next sorted job of the optical-depth walks,
// [26] and [27] crossings and deposits of the queued walks, [28] next chunk
// of the deposit walks, [29] a package beyond the attached gradient's
// workspace, [30] crossings of its peel rays' deposit walks.
constexpr int kJobCounter = 24, kKeyCounter = 25, kQueueCrossings = 26, kDepCounter = 28, kAttOverflow = 29,
              kAttDepCrossings = 30;
// Deposit-queue slots are reserved per wavefront in chunks (one global
// atomic per chunk); slots a wavefront reserved but did not fill are marked
// with kNoKey when it exits, and the sort skips them.
constexpr unsigned kJobChunk = 256, kNoKey = 0xffffffffu;

// The walk deposits -- the forward's absorbed light, the adjoint's gradient
// terms -- leave through an LDS transpose.  The deposits of kDepBlocks walk
// blocks are staged per wavefront first: entry kDepPer * lane + kBlockWalk * b
// + d holds lane `lane`'s deposit of sub-step d of staged block b (index -1:
// none), written by the walk itself (LifeMem::walk_deposit).  The
// flush's atomic instruction k then takes entries 64 k + lane, so the kDepPer
// deposits of one walker -- consecutive cells of its walk, often in one
// segment of the bricked array -- go out in adjacent lanes of one
// instruction, which the memory pipeline merges into one request per
// segment.  Global atomics are executed at the memory side at a fixed request
// rate, so fewer requests is what counts, and a longer run of one walker's
// cells splits into fewer segments per deposit.  Called by every lane of the
// wavefront (uniform control flow).
constexpr int kDepBlocks = 4, kDepPer = kDepBlocks * kBlockWalk;
static_assert(64 % kDepPer == 0, "a flush instruction holds whole walkers");

// Issues the nb staged blocks (entries of later blocks are stale and skipped:
// entry 64 k + lane is deposit (lane mod kDepPer) of its walker).
__device__ __forceinline__ void flush_deposits(int nb, double* tally, long long* sidx, double* sval) {
  const int lane = __lane_id();
  const bool fresh = (lane % kDepPer) < nb * kBlockWalk;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
  for (int k = 0; k < kDepPer; ++k) {
    const long long i = sidx[64 * k + lane];
    if (fresh && i >= 0) atomic_add_f64(tally + i, sval[64 * k + lane]);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Per-wavefront reservoir slots in LDS; lane 0 of each wavefront empties its
// slot before the wavefront's first fetch.
__device__ __forceinline__ unsigned long long* wave_reservoir(unsigned long long (&slots)[kWavesPerBlock][2]) {
  unsigned long long* r = slots[threadIdx.x / 64];
  if (__lane_id() == 0) r[0] = r[1] = 0;
  return r;
}

// ---------------------------------------------------------------------------
// Device memory accessors.

template <typename R, int GK, bool INST>
struct LifeMem {
  static constexpr int kGrid = GK;
  // the full variant: instruments other than frames (SED, camera) and the
  // optics and absorbed-tally gradients; the lean one compiles them out
  static constexpr bool kInst = INST;
  const R* __restrict__ rho_;
  const RunParams& P;
  unsigned long long* res;
  unsigned long long* job_res;
  __device__ R rho(int c) const { return rho_[c]; }
  __device__ const DetDev& det(int d) const { return P.det[d]; }
  __device__ const LamDev& lam(int l) const { return P.lam[l]; }
  __device__ const SrcDev& src(int s) const { return P.src[s]; }
  __device__ double adj(long long i) const { return P.adj[i]; }
  __device__ double adj_abs(long long i) const { return P.adj_abs[i]; }
  __device__ void add_image(long long i, double v) const { atomic_add_f64(P.images + i, v); }
  __device__ void add_absorbed(long long i, double v) const { atomic_add_f64(P.absorbed + i, v); }
  __device__ void add_grad(int i, double v) const { atomic_add_f64(P.grad + i, v); }
  // walk deposits: this lane's LDS staging entries of the current walk block
  long long* sidx;
  double* sval;
  int dbase;
  __device__ void stage_clear(int b) {
    dbase = kDepPer * __lane_id() + kBlockWalk * b;
#pragma unroll
    for (int d = 0; d < kBlockWalk; ++d) sidx[dbase + d] = -1ll;
  }
  template <bool ADJ>
  __device__ void walk_deposit(int d, long long i, double v) const {
    sidx[dbase + d] = i;
    sval[dbase + d] = v;
  }
  __device__ unsigned long long fetch() const { return wave_fetch(P.work, res, 64); }
  __device__ unsigned long long job_slot() const { return wave_fetch(P.work + kJobCounter, job_res, kJobChunk); }
  // event scratch of the adjoint: [ev_max][ev_k][n_chunk], then [n_chunk]
  __device__ double ev_load(int slot, int e, int k) const {
    return P.evs[((size_t)e * P.ev_k + k) * P.n_chunk + slot];
  }
  __device__ void ev_store(int slot, int e, int k, double v) const {
    P.evs[((size_t)e * P.ev_k + k) * P.n_chunk + slot] = v;
  }
  __device__ double ev_load_beyond(int slot) const { return P.evs[(size_t)P.ev_max * P.ev_k * P.n_chunk + slot]; }
  __device__ void opt_store(int slot, double ga, double gg, double gl, int src) const {
    P.gpart[slot] = ga;
    P.gpart[P.n_chunk + slot] = gg;
    P.gpart[2 * P.n_chunk + slot] = gl;
    P.gpart[3 * P.n_chunk + slot] = (double)src;
  }
  __device__ void ev_add_beyond(int slot, double v) const {
    atomic_add_f64(P.evs + (size_t)P.ev_max * P.ev_k * P.n_chunk + slot, v);
  }
  __device__ void store_job(unsigned long long slot, const double r[3], double v, long long ii, unsigned key,
                            unsigned sub, unsigned item, int e, int d, unsigned lam) const {
    PeelJob& J = P.jobs[slot];
    J.r[0] = r[0];
    J.r[1] = r[1];
    J.r[2] = r[2];
    J.v = v;
    J.ii = ii;
    J.slot = item;
    J.lam = lam;
    J.e = (unsigned short)e;
    J.d = (unsigned char)d;
    P.keys[slot] = key | (sub << 16);  // the sort reads these words only, not the 56-byte rays
  }
  // the forward run's tape: T of the leg after event e, C and the image
  // index of its peel-off into frame d (work item = item0 + slot)
  __device__ void tape_leg(int slot, int e, double T) const {
    if (e < P.tape_ev)
      P.tape[(size_t)e * (1 + P.n_det) * P.tape_n + P.item0 + slot] = T;
    else
      atomicOr(P.tape_over, 1u);
  }
  __device__ void tape_peel(int slot, int e, int d, double C, long long ii) const {
    if (e < P.tape_ev) {
      const size_t item = P.item0 + slot;
      P.tape[((size_t)e * (1 + P.n_det) + 1 + d) * P.tape_n + item] = C;
      P.tape_pix[((size_t)e * P.n_det + d) * P.tape_n + item] = (unsigned)ii;
    } else {
      atomicOr(P.tape_over, 1u);
    }
  }
  __device__ void flush_counts(unsigned a, unsigned b, unsigned c, unsigned d) const {
    atomicAdd(P.xstats + 0, (unsigned long long)a);
    atomicAdd(P.xstats + 1, (unsigned long long)b);
    atomicAdd(P.xstats + 2, (unsigned long long)c);
    atomicAdd(P.xstats + 6, (unsigned long long)d);
  }
};

template <typename R, int GK>
struct TraceMem {
  static constexpr int kGrid = GK;
  const R* __restrict__ rho_;
  const TraceParams& P;
  unsigned long long* res;
  __device__ R rho(int c) const { return rho_[c]; }
  __device__ unsigned long long fetch() const { return wave_fetch(P.work, res, 256); }
  __device__ void ray(long long q, double o[3], double k[3]) const {
    for (int a = 0; a < 3; ++a) {
      o[a] = P.origin[3 * q + a];
      k[a] = P.dir[3 * q + a];
    }
  }
  __device__ void set_tau(long long q, double t) const { P.tau[q] = t; }
  __device__ void set_nseg(long long q, int n) const {
    if (P.n_seg) P.n_seg[q] = n;
  }
  __device__ void store_seg(long long q, int j, int cell, double len) const {
    P.seg_cell[q * P.max_seg + j] = brick_to_linear(P.G, cell);
    P.seg_len[q * P.max_seg + j] = len;
  }
};

template <typename R, int GK>
struct PeelMem {
  static constexpr int kGrid = GK;
  const R* __restrict__ rho_;
  const PeelParams& P;
  unsigned long long* res;
  __device__ R rho(int c) const { return rho_[c]; }
  __device__ unsigned long long fetch() const { return wave_fetch(P.work, res, 256); }
  __device__ const DetDev& det(int d) const { return P.det[d]; }
  __device__ void position(long long e, double r[3]) const {
    for (int a = 0; a < 3; ++a) r[a] = P.pos[3 * e + a];
  }
  __device__ bool dir_in(long long e, double k[3]) const {
    if (!P.dir_in) return false;
    for (int a = 0; a < 3; ++a) k[a] = P.dir_in[3 * e + a];
    return true;
  }
  __device__ double weight(long long e) const { return P.w[e]; }
  __device__ void add_image(long long i, double v) const { atomic_add_f64(P.images + i, v); }
};

// ---------------------------------------------------------------------------
// Kernels.

// The life-cycle kernel body; k_life (FP32 walk) and k_life64 (FP64 walk)
// launch it, once per grid kind (GK, kGrid*) and with or without the
// handling of instruments other than frames -- SED instruments, cameras and
// their walks to the eye -- and of the adjoint's optics and absorbed-tally
// gradients (INST).  Every variant asks for two wavefronts per SIMD, which
// its register use could otherwise just miss (one accumulation register
// beyond 256 halves the occupancy).
template <typename R, bool ADJ, int GK, bool INST>
__device__ __forceinline__ void life_body(const RunParams& P) {
  __shared__ unsigned long long slots[kWavesPerBlock][2], job_slots[kWavesPerBlock][2];
  __shared__ long long dep_idx[kWavesPerBlock][64 * kDepPer];
  __shared__ double dep_val[kWavesPerBlock][64 * kDepPer];
  const int wave = threadIdx.x / 64;
  LifeMem<R, GK, INST> M{static_cast<const R*>(P.rho), P, wave_reservoir(slots), wave_reservoir(job_slots),
                         dep_idx[wave], dep_val[wave], 0};
  Lane<R> L;
  lane_init(L);
  int staged = 0;  // walk blocks of deposits staged in LDS (wavefront-uniform)
  double* const tally = ADJ ? P.grad : P.absorbed;
  for (;;) {
    lane_events<R, ADJ>(L, P, M);
    const unsigned long long live = __ballot(!L.done);
    if (live == 0ull) break;
    const int n_live = __popcll(live);
    for (;;) {
      const int n_act = __popcll(__ballot(L.ry.active));
      if (n_act == 0 || n_live - n_act >= P.batch) break;
      M.stage_clear(staged);
      const bool put = L.ry.active && lane_step<R, ADJ>(L, P, M);
      if (__ballot(put)) {
        if (++staged == kDepBlocks) {
          flush_deposits(staged, tally, dep_idx[wave], dep_val[wave]);
          staged = 0;
        }
      }
    }
  }
  if (staged) flush_deposits(staged, tally, dep_idx[wave], dep_val[wave]);
  if (P.jobs) {  // unfilled reserved queue slots
    const unsigned long long lo = M.job_res[0], hi = M.job_res[1] < P.job_cap ? M.job_res[1] : P.job_cap;
    for (unsigned long long q = lo + __lane_id(); q < hi; q += 64) P.keys[q] = kNoKey;
  }
  const double s_abs = wave_sum(L.s_abs), s_esc = wave_sum(L.s_esc), s_trunc = wave_sum(L.s_trunc);
  const unsigned long long a0 = wave_sum_u64(L.x_path), a1 = wave_sum_u64(L.x_loc), a2 = wave_sum_u64(L.x_peel),
                           a3 = wave_sum_u64(L.n_ev), a4 = wave_sum_u64(L.n_pk), a5 = wave_sum_u64(L.n_pl),
                           a6 = wave_sum_u64(L.n_dep);
  if (__lane_id() == 0) {
    atomic_add_f64(P.dstats + 0, s_abs);
    atomic_add_f64(P.dstats + 1, s_esc);
    atomic_add_f64(P.dstats + 2, s_trunc);
    atomicAdd(P.xstats + 0, a0);
    atomicAdd(P.xstats + 1, a1);
    atomicAdd(P.xstats + 2, a2);
    atomicAdd(P.xstats + 3, a3);
    atomicAdd(P.xstats + 4, a4);
    atomicAdd(P.xstats + 5, a5);
    atomicAdd(P.xstats + 6, a6);
  }
}

// Every variant asks for two wavefronts per SIMD: left free, the compiler
// took the lean rectilinear adjoint to 256 VGPRs and an AGPR, one wavefront
// per SIMD (PowCub adjoint life kernel 176 -> 301 ms); with the attribute
// every variant fits without spills (236-251 VGPRs lean).
template <typename R, bool ADJ, int GK, bool INST>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) k_life(const RunParams P) {
  life_body<R, ADJ, GK, INST>(P);
}

template <bool ADJ, int GK, bool INST>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2))) k_life64(const RunParams P) {
  life_body<double, ADJ, GK, INST>(P);
}

template <typename R, int GK>
__global__ void __launch_bounds__(kBlock) k_trace(const TraceParams P) {
  __shared__ unsigned long long slots[kWavesPerBlock][2];
  TraceMem<R, GK> M{static_cast<const R*>(P.rho), P, wave_reservoir(slots)};
  TraceLane<R> L;
  trace_init(L);
  for (;;) {
    trace_events(L, P, M);
    const unsigned long long live = __ballot(!L.done);
    if (live == 0ull) break;
    const int n_live = __popcll(live);
    for (;;) {
      const int n_act = __popcll(__ballot(L.ry.active));
      if (n_act == 0 || n_live - n_act >= P.batch) break;
      if (L.ry.active) trace_step(L, P, M);
    }
  }
  const unsigned long long total = wave_sum_u64(L.total), overflow = wave_sum_u64(L.overflow);
  if (__lane_id() == 0) {
    atomicAdd(P.counters + 0, total);
    if (overflow) atomicAdd(P.counters + 1, overflow);
  }
}

template <typename R, int GK>
__global__ void __launch_bounds__(kBlock) k_peel(const PeelParams P) {
  __shared__ unsigned long long slots[kWavesPerBlock][2];
  PeelMem<R, GK> M{static_cast<const R*>(P.rho), P, wave_reservoir(slots)};
  PeelLane<R> L;
  peel_init(L);
  for (;;) {
    peel_events(L, P, M);
    const unsigned long long live = __ballot(!L.done);
    if (live == 0ull) break;
    const int n_live = __popcll(live);
    for (;;) {
      const int n_act = __popcll(__ballot(L.ry.active));
      if (n_act == 0 || n_live - n_act >= P.batch) break;
      if (L.ry.active) peel_step(L, P, M);
    }
  }
}

// ---------------------------------------------------------------------------
// Queued peel rays.  The life kernel of the forward run and pass A of the
// adjoint queue each peel ray of each event (origin, W Phi / D^2, pixel,
// frame) instead of walking it.  A counting sort by key (k_hist, a scan,
// k_scatter) orders the queue by frame and by image tile in Morton order, so
// any run of consecutive sorted rays is a compact patch of one frame:
// parallel rays a few cells apart that cross one narrow bundle of cells.
// k_peeltau walks each ray once for its optical depth, in a lean kernel with
// many waves per SIMD whose neighbouring lanes read the same lines, and adds
// C = v e^-tau to its pixel (forward) or keeps q = (dL/dI) C for pass B
// (adjoint).  In the adjoint, k_peeldep hands runs of sorted rays (chunks)
// to workgroups and walks each ray with q != 0 once more, without density
// loads, to deposit -q kappa l; the deposits are summed per cell in an LDS
// hash table and each distinct cell goes to the gradient with one global
// atomic.  Global atomics execute at the memory side at a fixed request
// rate, so this replaces one atomic per crossing by about one per cell and
// chunk.

// Queue slots handed out (the counter may have run past the capacity).
__device__ __forceinline__ unsigned long long queued_jobs(const unsigned long long* ctr, unsigned long long cap) {
  const unsigned long long n = ctr[kJobCounter];
  return n < cap ? n : cap;
}

// The sort cuts the queue into kSortBlocks equal parts, one per workgroup.
// k_hist counts each part's tile keys in LDS and writes the counts to
// column b of the key-major matrix counts[key][kSortBlocks]; the exclusive
// scan of that matrix gives each (key, part) its first sorted position;
// k_scatter starts an LDS counter per key there and hands positions out to
// the part's rays, writing each ray's index and second key.  k_refine then
// sorts each tile's run by the second key (the pixel inside the tile, then
// the depth of the ray's origin), one workgroup per tile, the same way.
// Slots a wavefront reserved but did not fill (kNoKey) are skipped.  No
// global atomics: LDS counters do the ranking; the order of rays with equal
// keys is arbitrary.  k_refine's counters hold two workgroups per compute
// unit, so its workgroups are wide: 1024 threads against 256 take the clumpy
// 512^3 forward's sorts from 72.4 to 67.2 ms (spiral 10.4 -> 9.3).
constexpr int kSortThreads = 1024, kSortBlocks = host::kSortBlocks, kRefineThreads = 1024,
              kSubKeys = 256 << kDepthBits;

static_assert(host::kSortKeys <= (1 << 16) && kSubKeys <= (1 << 16), "a ray's keys share one word: key | sub << 16");

__device__ __forceinline__ void sort_part(unsigned long long n, unsigned long long& lo, unsigned long long& hi) {
  const unsigned long long per = (n + kSortBlocks - 1) / kSortBlocks;
  lo = blockIdx.x * per;
  hi = lo + per < n ? lo + per : n;
}

__global__ void __launch_bounds__(kSortThreads) k_hist(const unsigned* __restrict__ keys,
                                                       const unsigned long long* __restrict__ ctr,
                                                       unsigned long long cap, int n_keys,
                                                       unsigned* __restrict__ counts) {
  __shared__ unsigned h[host::kSortKeys];
  for (int i = threadIdx.x; i < n_keys; i += kSortThreads) h[i] = 0u;
  __syncthreads();
  unsigned long long lo, hi;
  sort_part(queued_jobs(ctr, cap), lo, hi);
  for (unsigned long long j = lo + threadIdx.x; j < hi; j += kSortThreads) {
    const unsigned w = keys[j];
    if (w != kNoKey) atomicAdd(h + (w & 0xffffu), 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n_keys; i += kSortThreads) counts[(size_t)i * kSortBlocks + blockIdx.x] = h[i];
}

// Runs of one first key at least this long skip the second level: its one
// workgroup per run would walk such a run alone, some 3 us per 256 rays (a
// point source's emission peel-offs all start at one place, one pixel and
// one depth: 1e7 rays, 33 ms), so k_scatter places their rays in the first
// level's order itself.  Shorter runs keep the second level, whose order
// the peel walks need (the clumpy disk's busiest tiles hold a few 1e5 rays
// per chunk; with a bound of 65536 its peel walks took 1052 ms, not 478).
// k_hot marks the long runs, one bit per key.
constexpr unsigned kHotRun = 1u << 21;
__global__ void __launch_bounds__(kSortThreads) k_hot(const unsigned* __restrict__ starts, int n_keys,
                                                      unsigned* __restrict__ hot) {
  const int w = blockIdx.x * kSortThreads + threadIdx.x;
  if (w >= (n_keys + 31) / 32) return;
  unsigned bits = 0;
  for (int b = 0; b < 32; ++b) {
    const int k = 32 * w + b;
    if (k < n_keys && starts[(size_t)(k + 1) * kSortBlocks] - starts[(size_t)k * kSortBlocks] >= kHotRun) bits |= 1u << b;
  }
  hot[w] = bits;
}

__global__ void __launch_bounds__(kSortThreads) k_scatter(const unsigned* __restrict__ keys,
                                                          const unsigned long long* __restrict__ ctr,
                                                          unsigned long long cap, int n_keys,
                                                          const unsigned* __restrict__ starts,
                                                          const unsigned* __restrict__ hot,
                                                          unsigned* __restrict__ idx, unsigned short* __restrict__ subs,
                                                          unsigned* __restrict__ perm) {
  __shared__ unsigned h[host::kSortKeys], hb[host::kSortKeys / 32];
  for (int i = threadIdx.x; i < n_keys; i += kSortThreads) h[i] = starts[(size_t)i * kSortBlocks + blockIdx.x];
  unsigned any = 0;
  for (int i = threadIdx.x; i < (n_keys + 31) / 32; i += kSortThreads) any |= hb[i] = hot[i];
  const bool some_hot = __syncthreads_or(any != 0u);
  unsigned long long lo, hi;
  sort_part(queued_jobs(ctr, cap), lo, hi);
  for (unsigned long long j = lo + threadIdx.x; j < hi; j += kSortThreads) {
    const unsigned w = keys[j];
    if (w != kNoKey) {
      const unsigned k = w & 0xffffu;
      const unsigned q = atomicAdd(h + k, 1u);
      idx[q] = (unsigned)j;
      subs[q] = (unsigned short)(w >> 16);
      if (some_hot && ((hb[k >> 5] >> (k & 31)) & 1u)) perm[q] = (unsigned)j;
    }
  }
}

// Exclusive scan of counts[0, n) into starts[0, n] (the total in starts[n])
// in three launches:
// k_scan_tiles scans tiles of kScanTile counts within each block and writes
// the tile totals, k_scan_top scans the totals in one block, k_scan_add adds
// each tile's offset.
constexpr int kScanThreads = 256, kScanPer = 8, kScanTile = kScanThreads * kScanPer, kTopThreads = 1024;

__device__ __forceinline__ unsigned block_exclusive_scan(unsigned v, unsigned* lds, unsigned* total) {
  const int t = threadIdx.x;
  lds[t] = v;
  __syncthreads();
  for (int off = 1; off < (int)blockDim.x; off <<= 1) {  // Hillis-Steele inclusive scan
    const unsigned u = t >= off ? lds[t - off] : 0u;
    __syncthreads();
    lds[t] += u;
    __syncthreads();
  }
  const unsigned incl = lds[t];
  *total = lds[blockDim.x - 1];
  __syncthreads();
  return incl - v;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const unsigned* __restrict__ counts,
                                                             unsigned* __restrict__ starts, unsigned* __restrict__ tiles,
                                                             long long n) {
  __shared__ unsigned lds[kScanThreads];
  const long long base = (long long)blockIdx.x * kScanTile + (long long)threadIdx.x * kScanPer;
  unsigned v[kScanPer], s = 0;
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    v[i] = base + i < n ? counts[base + i] : 0u;
    s += v[i];
  }
  unsigned total;
  unsigned run = block_exclusive_scan(s, lds, &total);
#pragma unroll
  for (int i = 0; i < kScanPer; ++i) {
    if (base + i < n) starts[base + i] = run;
    run += v[i];
  }
  if (threadIdx.x == 0) tiles[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kTopThreads) k_scan_top(unsigned* __restrict__ tiles, long long n_tiles,
                                                          unsigned* __restrict__ starts, long long n) {
  __shared__ unsigned lds[kTopThreads];
  const long long per = (n_tiles + kTopThreads - 1) / kTopThreads;
  const long long lo = threadIdx.x * per, hi = lo + per < n_tiles ? lo + per : n_tiles;
  unsigned s = 0;
  for (long long i = lo; i < hi; ++i) s += tiles[i];
  unsigned total;
  unsigned run = block_exclusive_scan(s, lds, &total);
  for (long long i = lo; i < hi; ++i) {
    const unsigned t = tiles[i];
    tiles[i] = run;
    run += t;
  }
  if (threadIdx.x == 0) starts[n] = total;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_add(unsigned* __restrict__ starts,
                                                           const unsigned* __restrict__ tiles, long long n) {
  const long long base = (long long)blockIdx.x * kScanTile;
  const unsigned off = tiles[blockIdx.x];
  for (int i = threadIdx.x; i < kScanTile; i += kScanThreads)
    if (base + i < n) starts[base + i] += off;
}

// Workgroup k sorts the run [starts of key k, starts of key k + 1) of idx
// by subs (the pixel inside the tile, then the depth) into perm.  Only the
// n_sub counters the frames' second keys can reach are cleared and scanned
// (a 128^2 frame has one-pixel tiles and 6-bit second keys: 64 of 16384).
__global__ void __launch_bounds__(kRefineThreads) k_refine(const unsigned* __restrict__ starts,
                                                           const unsigned* __restrict__ idx,
                                                           const unsigned short* __restrict__ subs,
                                                           unsigned* __restrict__ perm, int n_sub) {
  __shared__ unsigned h[kSubKeys], scan[kRefineThreads];
  const unsigned lo = starts[(size_t)blockIdx.x * kSortBlocks], hi = starts[(size_t)(blockIdx.x + 1) * kSortBlocks];
  if (hi - lo <= 1u) {
    if (hi > lo && threadIdx.x == 0) perm[lo] = idx[lo];
    return;
  }
  if (hi - lo >= kHotRun) return;  // placed by k_scatter
  for (int i = threadIdx.x; i < n_sub; i += kRefineThreads) h[i] = 0u;
  __syncthreads();
  for (unsigned i = lo + threadIdx.x; i < hi; i += kRefineThreads) atomicAdd(h + subs[i], 1u);
  __syncthreads();
  // thread t scans counters [t per, (t + 1) per) (n_sub and the threads are powers of two)
  const int per = n_sub >= kRefineThreads ? n_sub / kRefineThreads : 1;
  const int c0 = threadIdx.x * per, c1 = c0 + per < n_sub ? c0 + per : n_sub;
  unsigned own = 0, total;
  for (int j = c0; j < c1; ++j) own += h[j];
  unsigned run = lo + block_exclusive_scan(own, scan, &total);
  for (int j = c0; j < c1; ++j) {
    const unsigned c = h[j];
    h[j] = run;
    run += c;
  }
  __syncthreads();
  for (unsigned i = lo + threadIdx.x; i < hi; i += kRefineThreads) perm[atomicAdd(h + subs[i], 1u)] = idx[i];
}

constexpr int kBundleThreads = 512;
constexpr int kTableBits = 12, kTable = 1 << kTableBits, kProbes = 4;
// Sorted rays per deposit-walk chunk: a longer run of neighbouring pixels
// shares more cells in the table before its flush; measured on the spiral's
// adjoint queue kernels, 76.0 / 73.1 / 74.2 / 78.3 ms for 1024 / 4096 / 8192 /
// 16384 rays (a table of 8192 entries costs workgroups per CU: 101 ms).
constexpr unsigned kChunk = 4096;

struct PeelJobParams {
  GridDev G;
  const void* rho;
  const DetDev* det;
  const LamDev* lam;
  int n_det;
  PeelJob* jobs;
  const unsigned* perm;      // sorted order of the queue
  // the adjoint's deposit weight of sorted ray i, as the low and high words
  // of a double at wlo[i], whi[i]: the sort's key and index arrays, free once
  // the order is known, written and read in sorted order
  unsigned* wlo;
  unsigned* whi;
  const unsigned* n_sorted;  // number of sorted rays
  double* images;            // forward
  const double* adj;
  double* grad;
  double* evs;  // event scratch of the chunk (see LifeMem)
  int ev_max, ev_k;
  unsigned long long n_chunk;
  unsigned long long* ctr;  // counter block of the call
  int batch;
  // forward run with a tape: C and the image index of each ray (see RunParams)
  double* tape;
  unsigned* tape_pix;
  unsigned* tape_over;
  int tape_ev;
  unsigned long long tape_n, item0;
  // adjoint from a tape: the deposit weight is the ray's own v (no
  // optical-depth walk ran)
  int direct_w;
};

// Density loads for the optical-depth walk; deposits of the deposit walk go
// into the workgroup's LDS table (open addressing, linear probing over at
// most kProbes slots); a deposit that finds no slot goes straight to the
// global tally.  LUT: cell addresses from the per-axis address terms in LDS
// (k_peeltau on regular grids whose three axes fit kLutCells entries).
template <typename R, int GK, bool LUT = false>
struct PeelJobMem {
  static constexpr int kGrid = GK;
  static constexpr bool kLut = LUT;
  const R* __restrict__ rho_;
  int* tk;
  double* tv;
  double* grad;
  const int* lut = nullptr;  // the table of lut_entry; axis a's index i at lut_first(G, a) + 1 + i
  int o1 = 0, o2 = 0;        // lut_first(G, 1) + 1, lut_first(G, 2) + 1
  __device__ R rho(int c) const { return rho_[c]; }
  __device__ int lut_addr(const int i[3]) const { return lut[i[0] + 1] + lut[o1 + i[1]] + lut[o2 + i[2]]; }
  __device__ void deposit(int cell, double v) const {
    const unsigned h = ((unsigned)cell * 2654435761u) >> (32 - kTableBits);
    for (int p = 0; p < kProbes; ++p) {
      const unsigned i = (h + (unsigned)p) & (kTable - 1);
      int k = __hip_atomic_load(tk + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      if (k == -1) {
        k = atomicCAS(tk + i, -1, cell);
        if (k == -1) k = cell;
      }
      if (k == cell) {
        __hip_atomic_fetch_add(tv + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        return;
      }
    }
    atomic_add_f64(grad + cell, v);
  }
};

// Adds each waiting contribution (has) to its pixel: neighbouring lanes of
// the sorted queue mostly share a pixel, so the wavefront sums the
// contributions of each distinct pixel and issues one atomic for it (rather
// than up to 64 atomics on one address, which the memory side executes one
// after another).  Called by every lane of the wavefront.
__device__ __forceinline__ void flush_images(bool& has, long long ii, double c, double* images) {
  unsigned long long pend = __ballot(has);
  while (pend) {
    const int leader = __ffsll((long long)pend) - 1;
    const long long lii = (long long)shfl_u64((unsigned long long)ii, leader);
    const bool mine = has && ii == lii;
    const double s = wave_sum(mine ? c : 0.0);
    if (__lane_id() == leader) atomic_add_f64(images + lii, s);
    if (mine) has = false;
    pend = __ballot(has);
  }
}

// The optical-depth walks of the sorted queue, one ray per lane in a lean
// persistent loop (no deposit table, so many waves per SIMD hide the density
// loads).  Forward: C = v e^-tau goes to the ray's pixel (flush_images).
// Adjoint: q = (dL/dI) v e^-tau goes to the event scratch, and the deposit
// weight -q kappa to the ray's sorted position (wlo, whi; 0: no deposit walk).
//
// LUT (regular grids): the workgroup first writes the table of per-axis
// address terms (lut_entry) into LDS; the walk then adds three entries per
// cell, a few vector instructions against the dozen of the shifts and
// multiplies, in a kernel whose walk is bound by instruction issue.
template <typename R, bool ADJ, int GK, bool INST, bool LUT>
__global__ void __launch_bounds__(kBlock) k_peeltau(const PeelJobParams P) {
  __shared__ unsigned long long slots[kWavesPerBlock][2];
  __shared__ int lut[LUT ? kLutCells : 1];
  unsigned long long* res = wave_reservoir(slots);
  PeelJobMem<R, GK, LUT> M{static_cast<const R*>(P.rho), nullptr, nullptr, P.grad};
  if constexpr (LUT) {
    const int tot = lut_cells(P.G);  // the launch checks tot <= kLutCells
    for (int t = (int)threadIdx.x; t < tot; t += (int)blockDim.x) lut[t] = lut_entry(P.G, t);
    __syncthreads();
    M.lut = lut;
    M.o1 = lut_first(P.G, 1) + 1;
    M.o2 = lut_first(P.G, 2) + 1;
  }
  const unsigned n_jobs = *P.n_sorted;
  unsigned long long nx = 0;
  Ray<R> ry;
  ry.active = false;
  ry.tau = R(0);
  bool done = false, pending = false, has = false;
  unsigned job = 0, pend_qi = 0;
  R kap = R(0);
  long long out_ii = 0;
  double out_c = 0.0;
  for (;;) {
    while (!ry.active && !done) {
      if (pending) {
        PeelJob& J = P.jobs[job];
        const double C = J.v * exp(-(double)ry.tau);
        if (!ADJ) {
          if (has) atomic_add_f64(P.images + out_ii, out_c);  // a second ray ended in this refill
          out_ii = J.ii;
          out_c = C;
          has = true;
          if (P.tape) {
            if (J.e < P.tape_ev) {
              const size_t item = P.item0 + J.slot;
              P.tape[((size_t)J.e * (1 + P.n_det) + 1 + J.d) * P.tape_n + item] = C;
              P.tape_pix[((size_t)J.e * P.n_det + J.d) * P.tape_n + item] = (unsigned)J.ii;
            } else {
              atomicOr(P.tape_over, 1u);
            }
          }
        } else {
          const double q = P.adj[J.ii] * C;
          if (J.e < P.ev_max)
            P.evs[((size_t)J.e * P.ev_k + 1 + J.d) * P.n_chunk + J.slot] = q;
          else
            atomic_add_f64(P.evs + (size_t)P.ev_max * P.ev_k * P.n_chunk + J.slot, q);
          const double w = -q * P.lam[J.lam].kappa;
          const unsigned long long wb = (unsigned long long)__double_as_longlong(w);
          P.wlo[pend_qi] = (unsigned)wb;
          P.whi[pend_qi] = (unsigned)(wb >> 32);
        }
        pending = false;
      }
      const unsigned long long qi = wave_fetch(P.ctr + kKeyCounter, res, 256);
      if (qi >= n_jobs) {
        done = true;
        break;
      }
      job = P.perm[qi];
      pend_qi = (unsigned)qi;
      const PeelJob& J = P.jobs[job];
      kap = (R)P.lam[J.lam].kappa;
      if constexpr (INST) {
        double kd[3], inv_d2, tmax;
        peel_geometry(P.det[J.d], J.r, kd, inv_d2, tmax);
        ray_begin<R, GK>(ry, P.G, J.r, kd, tmax);
      } else {
        ray_begin<R, GK>(ry, P.G, J.r, P.det[J.d].kd);
      }
      pending = true;
    }
    if (!ADJ) flush_images(has, out_ii, out_c, P.images);
    const unsigned long long live = __ballot(!done);
    if (live == 0ull) break;
    const int n_live = __popcll(live);
    for (;;) {
      const int n_act = __popcll(__ballot(ry.active));
      if (n_act == 0 || n_live - n_act >= P.batch) break;
      if (ry.active) nx += tau_step<R, decltype(M), INST>(ry, P.G, kap, M);
    }
  }
  const unsigned long long wsum = wave_sum_u64(nx);
  if (__lane_id() == 0 && wsum) atomicAdd(P.ctr + kQueueCrossings, wsum);
}

// The deposit walks of the sorted queue: chunks of consecutive sorted jobs
// per workgroup, deposits summed per cell in the LDS table, one global
// atomic per distinct cell and chunk.  Jobs whose weight is 0 are skipped.
template <typename R, int GK, bool INST>
__global__ void __launch_bounds__(kBundleThreads) k_peeldep(const PeelJobParams P) {
  __shared__ int tk[kTable];
  __shared__ double tv[kTable];
  __shared__ unsigned s_begin, s_end, s_next;
  for (int i = threadIdx.x; i < kTable; i += kBundleThreads) {
    tk[i] = -1;
    tv[i] = 0.0;
  }
  const PeelJobMem<R, GK> M{static_cast<const R*>(P.rho), tk, tv, P.grad};
  const unsigned n_jobs = *P.n_sorted;
  unsigned long long nd = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      const unsigned long long b = atomicAdd(P.ctr + kDepCounter, 1ull) * kChunk;
      s_begin = s_next = b < n_jobs ? (unsigned)b : n_jobs;
      s_end = b + kChunk < n_jobs ? (unsigned)(b + kChunk) : n_jobs;
    }
    __syncthreads();
    const unsigned end = s_end;
    if (s_begin >= end) break;  // s_begin and s_end change only after the closing barrier
    Ray<R> ry;
    ry.active = false;
    bool done = false;
    double w = 0.0;
    for (;;) {
      while (!ry.active && !done) {
        const unsigned qi = atomicAdd(&s_next, 1u);
        if (qi >= end) {
          done = true;
          break;
        }
        w = P.direct_w ? P.jobs[P.perm[qi]].v
                       : __longlong_as_double((long long)(((unsigned long long)P.whi[qi] << 32) | P.wlo[qi]));
        if (w != 0.0) {
          const PeelJob& J = P.jobs[P.perm[qi]];
          if constexpr (INST) {
            double kd[3], inv_d2, tmax;
            peel_geometry(P.det[J.d], J.r, kd, inv_d2, tmax);
            ray_begin<R, GK>(ry, P.G, J.r, kd, tmax);
          } else {
            ray_begin<R, GK>(ry, P.G, J.r, P.det[J.d].kd);
          }
        }
      }
      const unsigned long long live = __ballot(!done);
      if (live == 0ull) break;
      const int n_live = __popcll(live);
      for (;;) {
        const int n_act = __popcll(__ballot(ry.active));
        if (n_act == 0 || n_live - n_act >= P.batch) break;
        if (ry.active) nd += bp_step<R, decltype(M), INST>(ry, P.G, w, M);
      }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kTable; i += kBundleThreads) {
      const int c = tk[i];
      if (c >= 0) {
        atomic_add_f64(P.grad + c, tv[i]);
        tk[i] = -1;
        tv[i] = 0.0;
      }
    }
    __syncthreads();
  }
  const unsigned long long dsum = wave_sum_u64(nd);
  if (__lane_id() == 0 && dsum) {
    atomicAdd(P.ctr + kQueueCrossings, dsum);
    atomicAdd(P.ctr + kQueueCrossings + 1, dsum);
  }
}

// ---------------------------------------------------------------------------
// The attached density gradient (mcrt_attached.hpp): one work item per lane,
// its forward sweep and its reverse sweep back to back, in FP64 arithmetic
// whatever the densities' storage (the FP32 path's densities are read as
// FP32 and widened).  A plain grid over
// the chunk's items -- each lane's work is one package's walks, done in
// order, so there is no state machine to interleave; the workspace keeps
// each item's events with the items of a chunk side by side, so lanes at the
// same event of their packages touch adjacent words.  Deposits go straight to
// the gradient as FP64 atomics.

template <typename S, int GK>
struct AttMem {
  static constexpr int kGrid = GK;
  const S* __restrict__ rho_;  // the densities as stored (FP32 or FP64), read as FP64
  const RunParams& P;
  __device__ double rho(int c) const { return (double)rho_[c]; }
  __device__ const DetDev& det(int d) const { return P.det[d]; }
  __device__ const LamDev& lam(int l) const { return P.lam[l]; }
  __device__ const SrcDev& src(int s) const { return P.src[s]; }
  __device__ double adj(long long i) const { return P.adj[i]; }
  __device__ void add_grad(int i, double v) const { atomic_add_f64(P.grad + i, v); }
  __device__ double att_ld(int slot, int e, int f) const {
    return P.evs[((size_t)e * kAttF + f) * P.n_chunk + slot];
  }
  __device__ void att_st(int slot, int e, int f, double v) const {
    P.evs[((size_t)e * kAttF + f) * P.n_chunk + slot] = v;
  }
  __device__ void att_over() const { atomicOr(P.work + kAttOverflow, 1ull); }
  // a peel ray's deposit walk of weight w into the peel-job queue (the
  // adjoint's sort keys; k_peeldep takes w as the ray's weight); false when
  // there is no queue or it is full
  unsigned long long* job_res;
  __device__ bool queue_deposit(const DetDev& D, int d, const double r[3], int pix, double w, long long ii,
                                unsigned item, int e, unsigned lam) const {
    if (!P.jobs) return false;
    const unsigned long long slot = wave_fetch(P.work + kJobCounter, job_res, kJobChunk);
    if (slot >= P.job_cap) return false;
    const int kp = key_pixel<true>(D, r, pix);
    PeelJob& J = P.jobs[slot];
    J.r[0] = r[0];
    J.r[1] = r[1];
    J.r[2] = r[2];
    J.v = w;
    J.ii = ii;
    J.slot = item;
    J.lam = lam;
    J.e = (unsigned short)(e < kEventSat ? e : kEventSat);
    J.d = (unsigned char)d;
    P.keys[slot] = tile_key(D, kp) | (sort_sub(D, kp, r, P.depth_drop) << 16);
    return true;
  }
};

// Persistent: a lane that has finished its package takes the next one from
// the chunk's work counter (packages differ widely in their number of
// events, and a wavefront of one package per lane lasts as long as its
// longest one).
template <typename S, int GK>
__global__ void __launch_bounds__(kBlock) k_attached(const RunParams P) {
  __shared__ unsigned long long slots[kWavesPerBlock][2], job_slots[kWavesPerBlock][2];
  unsigned long long* const res = wave_reservoir(slots);
  AttMem<S, GK> M{static_cast<const S*>(P.rho), P, wave_reservoir(job_slots)};
  AttCounts c;
  for (;;) {
    const unsigned long long k = wave_fetch(P.work, res, 64);
    if (k >= P.n_chunk) break;
    attached_item<double>(P, M, P.item0 + k, (int)k, c);
  }
  if (P.jobs) {  // unfilled reserved queue slots
    const unsigned long long lo = M.job_res[0], hi = M.job_res[1] < P.job_cap ? M.job_res[1] : P.job_cap;
    for (unsigned long long q = lo + __lane_id(); q < hi; q += 64) P.keys[q] = kNoKey;
  }
  const double s_abs = wave_sum(c.s_abs), s_esc = wave_sum(c.s_esc), s_trunc = wave_sum(c.s_trunc);
  const unsigned long long a0 = wave_sum_u64(c.x_path), a1 = wave_sum_u64(c.x_loc), a2 = wave_sum_u64(c.x_peel),
                           a3 = wave_sum_u64(c.n_ev), a4 = wave_sum_u64(c.n_pk), a5 = wave_sum_u64(c.n_pl),
                           a6 = wave_sum_u64(c.n_dep), a7 = wave_sum_u64(c.x_dep);
  if (__lane_id() == 0) {
    atomicAdd(P.work + kAttDepCrossings, a7);
    atomic_add_f64(P.dstats + 0, s_abs);
    atomic_add_f64(P.dstats + 1, s_esc);
    atomic_add_f64(P.dstats + 2, s_trunc);
    atomicAdd(P.xstats + 0, a0);
    atomicAdd(P.xstats + 1, a1);
    atomicAdd(P.xstats + 2, a2);
    atomicAdd(P.xstats + 3, a3);
    atomicAdd(P.xstats + 4, a4);
    atomicAdd(P.xstats + 5, a5);
    atomicAdd(P.xstats + 6, a6);
  }
}

__global__ void k_zero(double* __restrict__ p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// Row-major densities -> bricked layout (padding cells 0); one thread per
// bricked cell, so the writes are contiguous.
template <typename R>
__global__ void k_brick(const R* __restrict__ src, R* __restrict__ dst, const GridDev G) {
  for (long long c = blockIdx.x * (long long)blockDim.x + threadIdx.x; c < G.ncell_pad;
       c += (long long)gridDim.x * blockDim.x) {
    int i[3];
    const bool in = brick_cell(G, (int)c, i);
    dst[c] = in ? src[i[0] + i[1] * G.stride[1] + i[2] * G.stride[2]] : R(0);
  }
}

// Library tally -> row-major [n_lambda][ncell]; one thread per row-major
// cell.  slots: the forward's absorbed tally [n_lambda][ntal], cell c at
// tally_slot(c); otherwise a bricked array [n_lambda][ncell_pad].
__global__ void k_unbrick(const double* __restrict__ src, double* __restrict__ dst, const GridDev G, int n_lambda,
                          bool slots) {
  const long long n = (long long)n_lambda * G.ncell;
  for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
    const long long l = q / G.ncell;
    const int m = (int)(q - l * G.ncell);
    int i[3];
    i[0] = m % G.n[0];
    const int t = m / G.n[0];
    i[1] = t % G.n[1];
    i[2] = t / G.n[1];
    const int c = brick_addr(G, i);
    dst[q] = slots ? src[l * G.ntal + tally_slot(G, c)] : src[l * G.ncell_pad + c];
  }
}

// The adjoint's event scratch of a chunk from the forward run's tape: per
// package (slot) and kept event, T of the leg after it and q = (dL/dI) C per
// frame; nothing lies beyond the kept events.  One thread per package: the
// tape and the scratch are both [event][entry][package], so neighbouring
// lanes read and write neighbouring words.
__global__ void k_tape_q(const double* __restrict__ tape, const unsigned* __restrict__ pix,
                         const double* __restrict__ adj, double* __restrict__ evs, unsigned long long item0,
                         unsigned long long n_chunk, unsigned long long tape_n, int ev_max, int n_det) {
  for (unsigned long long slot = blockIdx.x * (unsigned long long)blockDim.x + threadIdx.x; slot < n_chunk;
       slot += (unsigned long long)gridDim.x * blockDim.x) {
    const unsigned long long item = item0 + slot;
    for (int e = 0; e < ev_max; ++e) {
      const size_t b = (size_t)e * (1 + n_det);
      evs[b * n_chunk + slot] = tape[b * tape_n + item];
      for (int d = 0; d < n_det; ++d) {
        const double C = tape[(b + 1 + d) * tape_n + item];
        evs[(b + 1 + d) * n_chunk + slot] = C != 0.0 ? adj[pix[((size_t)e * n_det + d) * tape_n + item]] * C : 0.0;
      }
    }
    evs[(size_t)ev_max * (1 + n_det) * n_chunk + slot] = 0.0;
  }
}

// ---------------------------------------------------------------------------
// Optics and luminosity gradients of a chunk: one workgroup per wavelength
// whose packages the chunk holds (block b: wavelength item0 / n_pkg + b)
// sums the pass-B sums of its packages (gpart [4][n_chunk]: sum q n, sum q
// score, sum q, source) and adds the gradients (optics_finish).
constexpr int kOptThreads = 256;

__global__ void __launch_bounds__(kOptThreads) k_grad_optics(const double* __restrict__ gpart,
                                                             unsigned long long item0, unsigned long long n_chunk,
                                                             unsigned long long n_pkg, int n_src,
                                                             const LamDev* __restrict__ lam,
                                                             const double* __restrict__ lums, int nl,
                                                             double* g_alb, double* g_g, double* g_lum) {
  const unsigned long long l = item0 / n_pkg + blockIdx.x;
  const unsigned long long b = l * n_pkg > item0 ? l * n_pkg : item0;
  const unsigned long long e = (l + 1) * n_pkg < item0 + n_chunk ? (l + 1) * n_pkg : item0 + n_chunk;
  double v[2 + MCRT_MAX_SOURCES];
  for (int q = 0; q < 2 + MCRT_MAX_SOURCES; ++q) v[q] = 0.0;
  for (unsigned long long it = b + threadIdx.x; it < e; it += kOptThreads) {
    const unsigned long long slot = it - item0;
    v[0] += gpart[slot];
    v[1] += gpart[n_chunk + slot];
    const double gl = gpart[2 * n_chunk + slot];
    const int src = (int)gpart[3 * n_chunk + slot];
#pragma unroll
    for (int q = 0; q < MCRT_MAX_SOURCES; ++q) v[2 + q] += q == src ? gl : 0.0;
  }
  __shared__ double red[kOptThreads];
  __shared__ double tot[2 + MCRT_MAX_SOURCES];
  for (int q = 0; q < 2 + n_src; ++q) {
    red[threadIdx.x] = v[q];
    __syncthreads();
    for (int w = kOptThreads / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) tot[q] = red[0];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    optics_finish(tot[0], tot[1], tot + 2, n_src, lam[l].albedo, lums + l, nl, g_alb, g_g, g_lum, (int)l, nl);
}

// ---------------------------------------------------------------------------
// Cell-source CDF: per wavelength row the exclusive prefix sums of the
// cells' luminosities x[row][0..n) into cum[row][0..n], cum[row][n] the
// total.  Tiles of kCdfTile cells; each thread sums kCdfPer consecutive cells
// in order, one thread of the tile adds the threads' sums in order, and one
// thread per row adds the tiles' sums in order.  Every entry is an offset
// plus a partial sum that the next entry extends by the cell's own
// luminosity, so cum never decreases and a cell of zero luminosity has
// cum[m + 1] == cum[m] exactly: it can never be drawn.  The tile kernel also
// flags a negative or non-finite luminosity.
constexpr int kCdfThreads = 256, kCdfPer = 8, kCdfTile = kCdfThreads * kCdfPer;

struct CdfTile {
  double part[kCdfPer];  // exclusive sums of the thread's cells
  double base;           // exclusive sum of the tile's earlier threads
  double total;          // sum of the tile
};

__device__ void cdf_tile(const double* __restrict__ row, long long n, long long tile, CdfTile& c, int* bad) {
  __shared__ double ts[kCdfThreads];
  __shared__ double tb[kCdfThreads + 1];
  const long long i0 = tile * kCdfTile + (long long)threadIdx.x * kCdfPer;
  double s = 0.0;
  bool ok = true;
  for (int k = 0; k < kCdfPer; ++k) {
    c.part[k] = s;
    const double v = i0 + k < n ? row[i0 + k] : 0.0;
    ok = ok && v >= 0.0 && v < INFINITY;
    s += v;
  }
  if (!ok) atomicOr(bad, 1);
  ts[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double acc = 0.0;
    for (int t = 0; t < kCdfThreads; ++t) {
      tb[t] = acc;
      acc += ts[t];
    }
    tb[kCdfThreads] = acc;
  }
  __syncthreads();
  c.base = tb[threadIdx.x];
  c.total = tb[kCdfThreads];
}

// One workgroup per (row, tile), blockIdx.x = row * n_tiles + tile.
__global__ void __launch_bounds__(kCdfThreads) k_cdf_tiles(const double* __restrict__ x, long long n, int n_tiles,
                                                           double* __restrict__ tile_sum, int* bad) {
  const long long row = blockIdx.x / n_tiles, tile = blockIdx.x - row * n_tiles;
  CdfTile c;
  cdf_tile(x + row * n, n, tile, c, bad);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = c.total;
}

// One thread per row: tile sums -> exclusive tile offsets, and the total.
__global__ void k_cdf_top(double* __restrict__ tile_sum, int n_tiles, int rows, double* __restrict__ cum, long long n,
                          double* __restrict__ totals) {
  const int row = blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= rows) return;
  double acc = 0.0;
  double* t = tile_sum + (long long)row * n_tiles;
  for (int q = 0; q < n_tiles; ++q) {
    const double v = t[q];
    t[q] = acc;
    acc += v;
  }
  cum[(long long)row * (n + 1) + n] = acc;
  totals[row] = acc;
}

__global__ void __launch_bounds__(kCdfThreads) k_cdf_apply(const double* __restrict__ x, long long n, int n_tiles,
                                                           const double* __restrict__ tile_off,
                                                           double* __restrict__ cum, int* bad) {
  const long long row = blockIdx.x / n_tiles, tile = blockIdx.x - row * n_tiles;
  CdfTile c;
  cdf_tile(x + row * n, n, tile, c, bad);
  const double off = tile_off[blockIdx.x];
  const long long i0 = tile * kCdfTile + (long long)threadIdx.x * kCdfPer;
  double* out = cum + row * (n + 1);
  for (int k = 0; k < kCdfPer; ++k)
    if (i0 + k < n) out[i0 + k] = off + (c.base + c.part[k]);
}

// ---------------------------------------------------------------------------
// Dust emission, one thread per cell; the table kernel fills ln P at the
// kDustTable + 1 points first.

__global__ void k_dust_table(DustDev D, double* __restrict__ lnP) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k <= kDustTable) lnP[k] = dust_table_entry(D, k);
}

template <typename R, int GK>
__global__ void __launch_bounds__(kBlock) k_dust_emission(DustParams P) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m < P.G.ncell) dust_cell<R, GK>(P, m);
}

}  // namespace mcrt

// ===========================================================================
// Host side: launches.

// Device block of trace_path_noalloc (see trace_impl): one per device, held
// until the process ends.
static __device__ __align__(256) unsigned char scratch[MCRT_NOALLOC_SCRATCH_BYTES];

namespace {

using namespace mcrt;
using host::fail;

#define HIPCHK(x)                                                                     \
  do {                                                                                \
    hipError_t e_ = (x);                                                              \
    if (e_ != hipSuccess) return fail(MCRT_EHIP, "%s: %s", #x, hipGetErrorString(e_)); \
  } while (0)

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

template <typename K>
int persistent_grid(K kernel, int blocks_per_cu, int* grid_out) {
  int dev = 0, cus = 0, nb = 0;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kBlock, 0));
  if (blocks_per_cu > 0) nb = blocks_per_cu;
  *grid_out = std::max(1, nb) * std::max(1, cus);
  return 0;
}

// Launches a persistent kernel with a full-occupancy grid of kBlock threads.
// (blocks_per_cu > 0: that many workgroups per compute unit instead.)
template <typename K, typename Params>
int launch_persistent(K kernel, const Params& P, hipStream_t st, int blocks_per_cu = 0) {
  int nblk = 0;
  if (int e = persistent_grid(kernel, blocks_per_cu, &nblk)) return e;
  hipLaunchKernelGGL(kernel, dim3(nblk), dim3(kBlock), 0, st, P);
  return 0;
}

// Launches the grid kind's variant of a persistent kernel.
template <typename Params, typename R, typename K>
int launch_by_kind(const Params& P, hipStream_t st, K regular, K rect, K tree, int blocks_per_cu = 0) {
  return launch_persistent(P.G.kind == kGridRect ? rect : (P.G.kind == kGridTree ? tree : regular), P, st,
                           blocks_per_cu);
}

// Workgroups per compute unit of the trace kernel.  Its rays are unrelated
// (no two lanes share lines), so fewer walkers thrash each XCD's 4 MB L2
// less: 4e6 random rays, 1.82 / 1.77 / 1.67 / 1.58e11 crossings/s on the
// spiral's grid with 2 / 3 / 4 / all it fits (6), 1.71 / 1.72 / 1.60 /
// 1.57e11 on the clumpy 512^3 grid.  The sorted peel rays are the opposite
// case: their lanes share lines, and their walk wants every wavefront it
// can get (clumpy: 612 ms at 5 workgroups per CU, 982 at 2).
constexpr int kTraceBlocksPerCu = 2;

unsigned stream_blocks(long long n) { return (unsigned)std::min<long long>((n + kBlock - 1) / kBlock, 16384); }

__global__ void k_zero_u32(unsigned* __restrict__ p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

int zero_fill(double* p, long long n, hipStream_t st) {
  if (!p || n <= 0) return 0;
  hipLaunchKernelGGL(k_zero, dim3(stream_blocks(n)), dim3(kBlock), 0, st, p, n);
  HIPCHK(hipGetLastError());
  return 0;
}

// Bricked copy of the caller's densities into dst (G.ncell_pad elements).
int brick_density(const GridDev& G, const void* rho, void* dst, bool f32, hipStream_t st) {
  if (f32)
    hipLaunchKernelGGL(k_brick<float>, dim3(stream_blocks(G.ncell_pad)), dim3(kBlock), 0, st,
                       static_cast<const float*>(rho), static_cast<float*>(dst), G);
  else
    hipLaunchKernelGGL(k_brick<double>, dim3(stream_blocks(G.ncell_pad)), dim3(kBlock), 0, st,
                       static_cast<const double*>(rho), static_cast<double*>(dst), G);
  HIPCHK(hipGetLastError());
  return 0;
}

int unbrick_tally(const GridDev& G, const double* src, double* dst, int n_lambda, bool slots, hipStream_t st) {
  hipLaunchKernelGGL(k_unbrick, dim3(stream_blocks((long long)n_lambda * G.ncell)), dim3(kBlock), 0, st, src, dst, G,
                     n_lambda, slots);
  HIPCHK(hipGetLastError());
  return 0;
}

// CDF of the cell source's luminosities cell_lum [n_lambda][ncell] (device)
// into cum [n_lambda][ncell + 1]; then the per-wavelength totals come to
// the host (the call waits for them) and set the package weights in pr.
int cell_cdf(const double* cell_lum, int nl, int ncell, double* cum, double* tile_sum, int n_tiles, double* totals,
             hipStream_t st, host::Prepared* pr, int n_src, const mcrt_source* sources, const mcrt_opts* opts) {
  int* bad = reinterpret_cast<int*>(totals + nl);
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned*>(bad), 1ll);
  const unsigned blocks = (unsigned)((long long)nl * n_tiles);
  hipLaunchKernelGGL(k_cdf_tiles, dim3(blocks), dim3(kCdfThreads), 0, st, cell_lum, (long long)ncell, n_tiles,
                     tile_sum, bad);
  hipLaunchKernelGGL(k_cdf_top, dim3((nl + 255) / 256), dim3(256), 0, st, tile_sum, n_tiles, nl, cum,
                     (long long)ncell, totals);
  hipLaunchKernelGGL(k_cdf_apply, dim3(blocks), dim3(kCdfThreads), 0, st, cell_lum, (long long)ncell, n_tiles,
                     tile_sum, cum, bad);
  HIPCHK(hipGetLastError());
  std::vector<double> tot(nl + 1);
  HIPCHK(hipMemcpyAsync(tot.data(), totals, sizeof(double) * nl + sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  int flag = 0;
  std::memcpy(&flag, tot.data() + nl, sizeof flag);
  if (flag) return fail(MCRT_EINVAL, "cell_lum holds a negative or non-finite luminosity");
  host::set_luminosities(*pr, n_src, sources, tot.data(), opts->n_packages);
  return 0;
}

// Per-call device memory (problem tables, zeroed counters, the bricked
// densities and tally): one allocation, ordered on the stream, released on
// the stream when the call returns.
struct DeviceBlock {
  unsigned char* ptr = nullptr;
  hipStream_t st = nullptr;
  ~DeviceBlock() {
    if (ptr) (void)hipFreeAsync(ptr, st);
  }
};

struct EventPair {
  hipEvent_t a = nullptr, b = nullptr, c = nullptr;
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (c) (void)hipEventDestroy(c);
  }
};

// HIP events recorded on the call's stream around the launches of each
// kind (only when the caller asks for statistics): the life-cycle kernel,
// the peel-ray sort, the optical-depth walks and the deposit walks.
enum SpanKind { kSpanLife = 0, kSpanSort, kSpanPeel, kSpanDep, kSpanKinds };
struct Spans {
  bool on = false;
  std::vector<hipEvent_t> ev[kSpanKinds];  // begin, end, begin, end, ...
  ~Spans() {
    for (auto& v : ev)
      for (hipEvent_t e : v) (void)hipEventDestroy(e);
  }
  int mark(int kind, hipStream_t st) {
    if (!on) return 0;
    hipEvent_t e = nullptr;
    HIPCHK(hipEventCreate(&e));
    ev[kind].push_back(e);
    HIPCHK(hipEventRecord(e, st));
    return 0;
  }
  // total milliseconds of the spans of one kind (after the stream has
  // finished them)
  double ms(int kind) const {
    double t = 0.0;
    for (size_t i = 0; i + 1 < ev[kind].size(); i += 2) {
      float x = 0.0f;
      if (hipEventElapsedTime(&x, ev[kind][i], ev[kind][i + 1]) == hipSuccess) t += x;
    }
    return t;
  }
};

// Device memory of the peel-ray queue: rays, their sorted order (and the
// order after the first sort pass with the second keys), the sort's count
// matrix (keys x kSortBlocks), its scan and the scan's tile totals.
constexpr size_t kQueueBytesPerRay = sizeof(PeelJob) + 3 * sizeof(unsigned) + sizeof(unsigned short);
struct PeelQueue {
  unsigned char* ptr = nullptr;
  hipStream_t st = nullptr;
  unsigned long long cap = 0;
  long long n_keys = 0;
  int n_sub = 0;  // counters of k_refine: 2^(width of the second keys)
  PeelJob* jobs = nullptr;
  unsigned *keys = nullptr, *perm = nullptr, *idx = nullptr, *counts = nullptr, *starts = nullptr, *tiles = nullptr;
  unsigned* hot = nullptr;  // bit k: key k's run is at least kHotRun rays (not refined)
  unsigned short* subs = nullptr;
  ~PeelQueue() {
    if (ptr) (void)hipFreeAsync(ptr, st);
  }
};

// Capacity per chunk of `chunk` packages: mcrt_opts.peel_queue, or by
// default 8 peel rays per package and frame (the typical package has fewer
// events; rays beyond the capacity are walked inline), at most 2^31 (the
// sort's positions are 32-bit) and a quarter of the free device memory.  The
// chunk follows the queue's byte budget, so the default capacity keeps its 8
// rays per package and frame.
int make_peel_queue(const mcrt_opts& o, const host::Prepared& pr, unsigned long long chunk, hipStream_t st,
                    PeelQueue& q) {
  q.st = st;
  q.n_keys = pr.n_keys;
  q.n_sub = 1 << pr.sub_bits;
  if (q.n_sub > kSubKeys) return fail(MCRT_EINVAL, "second sort keys of %d bits exceed the sort's counters", pr.sub_bits);
  unsigned long long cap;
  if (o.peel_queue > 0) {
    cap = (unsigned long long)o.peel_queue;
  } else {
    cap = chunk * (unsigned long long)pr.P.n_det * 8ull;
    cap = std::min(std::max(cap, 1ull << 16), 1ull << 31);
    size_t free_b = 0, total_b = 0;
    HIPCHK(hipMemGetInfo(&free_b, &total_b));
    cap = std::min<unsigned long long>(cap, free_b / 4 / kQueueBytesPerRay);
    if (cap == 0) return 0;
  }
  const size_t n_cnt = (size_t)q.n_keys * kSortBlocks;
  const size_t off_keys = align256(sizeof(PeelJob) * cap);
  const size_t off_perm = off_keys + align256(sizeof(unsigned) * cap);
  const size_t off_idx = off_perm + align256(sizeof(unsigned) * cap);
  const size_t off_subs = off_idx + align256(sizeof(unsigned) * cap);
  const size_t off_cnt = off_subs + align256(sizeof(unsigned short) * cap);
  const size_t off_start = off_cnt + align256(sizeof(unsigned) * n_cnt);
  const size_t off_tiles = off_start + align256(sizeof(unsigned) * (n_cnt + 1));
  const size_t off_hot = off_tiles + align256(sizeof(unsigned) * (n_cnt / kScanTile + 1));
  const size_t bytes = off_hot + align256(sizeof(unsigned) * (host::kSortKeys / 32));
  HIPCHK(hipMallocAsync(reinterpret_cast<void**>(&q.ptr), bytes, st));
  q.cap = cap;
  q.jobs = reinterpret_cast<PeelJob*>(q.ptr);
  q.keys = reinterpret_cast<unsigned*>(q.ptr + off_keys);
  q.perm = reinterpret_cast<unsigned*>(q.ptr + off_perm);
  q.idx = reinterpret_cast<unsigned*>(q.ptr + off_idx);
  q.subs = reinterpret_cast<unsigned short*>(q.ptr + off_subs);
  q.counts = reinterpret_cast<unsigned*>(q.ptr + off_cnt);
  q.starts = reinterpret_cast<unsigned*>(q.ptr + off_start);
  q.tiles = reinterpret_cast<unsigned*>(q.ptr + off_tiles);
  q.hot = reinterpret_cast<unsigned*>(q.ptr + off_hot);
  return 0;
}

// Zeroes counter words [w, w + n) of the call's counter block.
int reset_counters(unsigned long long* ctr, int w, int n, hipStream_t st) {
  return zero_fill(reinterpret_cast<double*>(ctr + w), n, st);
}

// The queue's walks: optical depth (and the image, forward), then the
// adjoint's deposit walks.
template <typename R, bool ADJ, int GK, bool INST>
int walk_peel_jobs(const PeelJobParams& J, hipStream_t st, Spans& sp) {
  if (!J.direct_w) {  // an adjoint from a tape has every ray's weight already: no optical-depth walk
    int nblk = 0;
    void (*kern)(PeelJobParams) = k_peeltau<R, ADJ, GK, INST, false>;
    if constexpr (GK == kGridRegular)
      if (lut_cells(J.G) <= kLutCells) kern = k_peeltau<R, ADJ, GK, INST, true>;
    PeelJobParams Jt = J;
    if ((long long)J.G.ncell_pad * (long long)sizeof(R) > kMallBytes) Jt.batch = kBatchQueueHbm;
    if (int e = persistent_grid(kern, 0, &nblk)) return e;
    if (int e = sp.mark(kSpanPeel, st)) return e;
    hipLaunchKernelGGL(kern, dim3(nblk), dim3(kBlock), 0, st, Jt);
    if (int e = sp.mark(kSpanPeel, st)) return e;
  }
  if (ADJ) {
    int dev = 0, cus = 0, nb = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_peeldep<R, GK, INST>, kBundleThreads, 0));
    if (int e = sp.mark(kSpanDep, st)) return e;
    hipLaunchKernelGGL((k_peeldep<R, GK, INST>), dim3(std::max(1, nb) * std::max(1, cus)), dim3(kBundleThreads), 0,
                       st, J);
    if (int e = sp.mark(kSpanDep, st)) return e;
  }
  HIPCHK(hipGetLastError());
  return 0;
}

// Sorts the chunk's queued peel rays by key and walks them.
template <typename R, bool ADJ>
int run_peel_jobs(const PeelQueue& q, const RunParams& P, unsigned long long* ctr, bool inst, hipStream_t st,
                  Spans& sp) {
  const long long n_cnt = q.n_keys * kSortBlocks;
  if (int e = sp.mark(kSpanSort, st)) return e;
  hipLaunchKernelGGL(k_hist, dim3(kSortBlocks), dim3(kSortThreads), 0, st, q.keys, ctr, q.cap, (int)q.n_keys,
                     q.counts);
  const long long n_tiles = (n_cnt + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)n_tiles), dim3(kScanThreads), 0, st, q.counts, q.starts, q.tiles,
                     n_cnt);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kTopThreads), 0, st, q.tiles, n_tiles, q.starts, n_cnt);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)n_tiles), dim3(kScanThreads), 0, st, q.starts, q.tiles, n_cnt);
  hipLaunchKernelGGL(k_hot, dim3((unsigned)((q.n_keys + 32 * kSortThreads - 1) / (32 * kSortThreads))),
                     dim3(kSortThreads), 0, st, q.starts, (int)q.n_keys, q.hot);
  hipLaunchKernelGGL(k_scatter, dim3(kSortBlocks), dim3(kSortThreads), 0, st, q.keys, ctr, q.cap, (int)q.n_keys,
                     q.starts, q.hot, q.idx, q.subs, q.perm);
  hipLaunchKernelGGL(k_refine, dim3((unsigned)q.n_keys), dim3(kRefineThreads), 0, st, q.starts, q.idx, q.subs, q.perm,
                     q.n_sub);
  HIPCHK(hipGetLastError());
  if (int e = sp.mark(kSpanSort, st)) return e;
  PeelJobParams J;
  J.G = P.G;
  J.rho = P.rho;
  J.det = P.det;
  J.lam = P.lam;
  J.n_det = P.n_det;
  J.jobs = q.jobs;
  J.perm = q.perm;
  J.wlo = q.keys;
  J.whi = q.idx;
  J.n_sorted = q.starts + n_cnt;
  J.images = P.images;
  J.adj = P.adj;
  J.grad = P.grad;
  J.evs = P.evs;
  J.ev_max = P.ev_max;
  J.ev_k = P.ev_k;
  J.n_chunk = P.n_chunk;
  J.ctr = ctr;
  J.batch = kBatchQueue;
  J.tape = P.tape;
  J.tape_pix = P.tape_pix;
  J.tape_over = P.tape_over;
  J.tape_ev = P.tape_ev;
  J.tape_n = P.tape_n;
  J.item0 = P.item0;
  J.direct_w = P.dep_jobs;
  if (inst) {  // instruments other than frames: walks that stop at a camera's eye
    switch (P.G.kind) {
      case kGridRect: return walk_peel_jobs<R, ADJ, kGridRect, true>(J, st, sp);
      case kGridTree: return walk_peel_jobs<R, ADJ, kGridTree, true>(J, st, sp);
      default: return walk_peel_jobs<R, ADJ, kGridRegular, true>(J, st, sp);
    }
  }
  switch (P.G.kind) {
    case kGridRect: return walk_peel_jobs<R, ADJ, kGridRect, false>(J, st, sp);
    case kGridTree: return walk_peel_jobs<R, ADJ, kGridTree, false>(J, st, sp);
    default: return walk_peel_jobs<R, ADJ, kGridRegular, false>(J, st, sp);
  }
}

template <typename R, bool ADJ, int GK, bool INST>
int life_grid_k(int blocks_per_cu, int* nblk) {
  if constexpr (std::is_same<R, double>::value)
    return persistent_grid(k_life64<ADJ, GK, INST>, blocks_per_cu, nblk);
  else
    return persistent_grid(k_life<R, ADJ, GK, INST>, blocks_per_cu, nblk);
}

template <typename R, bool ADJ, bool INST>
int life_grid_c(int kind, int blocks_per_cu, int* nblk) {
  switch (kind) {
    case kGridRect: return life_grid_k<R, ADJ, kGridRect, INST>(blocks_per_cu, nblk);
    case kGridTree: return life_grid_k<R, ADJ, kGridTree, INST>(blocks_per_cu, nblk);
    default: return life_grid_k<R, ADJ, kGridRegular, INST>(blocks_per_cu, nblk);
  }
}

template <typename R, bool ADJ>
int life_grid(int kind, bool inst, int blocks_per_cu, int* nblk) {
  return inst ? life_grid_c<R, ADJ, true>(kind, blocks_per_cu, nblk)
             : life_grid_c<R, ADJ, false>(kind, blocks_per_cu, nblk);
}

template <typename R, bool ADJ, int GK, bool INST>
void launch_life_k(const RunParams& P, int nblk, hipStream_t st) {
  if constexpr (std::is_same<R, double>::value)
    hipLaunchKernelGGL((k_life64<ADJ, GK, INST>), dim3(nblk), dim3(kBlock), 0, st, P);
  else
    hipLaunchKernelGGL((k_life<R, ADJ, GK, INST>), dim3(nblk), dim3(kBlock), 0, st, P);
}

template <typename R, bool ADJ, bool INST>
void launch_life_c(const RunParams& P, int nblk, hipStream_t st) {
  if (P.G.kind == kGridRect)
    launch_life_k<R, ADJ, kGridRect, INST>(P, nblk, st);
  else if (P.G.kind == kGridTree)
    launch_life_k<R, ADJ, kGridTree, INST>(P, nblk, st);
  else
    launch_life_k<R, ADJ, kGridRegular, INST>(P, nblk, st);
}

// The attached gradient's kernel over one chunk (its work counter reset by
// the caller): a persistent grid; f32: the densities are stored in FP32.
int launch_attached(const RunParams& P, bool f32, hipStream_t st) {
  const int kind = P.G.kind;
  int e;
  if (f32)
    e = kind == kGridRect   ? launch_persistent(k_attached<float, kGridRect>, P, st)
        : kind == kGridTree ? launch_persistent(k_attached<float, kGridTree>, P, st)
                            : launch_persistent(k_attached<float, kGridRegular>, P, st);
  else
    e = kind == kGridRect   ? launch_persistent(k_attached<double, kGridRect>, P, st)
        : kind == kGridTree ? launch_persistent(k_attached<double, kGridTree>, P, st)
                            : launch_persistent(k_attached<double, kGridRegular>, P, st);
  if (e) return e;
  HIPCHK(hipGetLastError());
  return 0;
}

template <typename R, bool ADJ>
int launch_life(const RunParams& P, bool inst, int nblk, hipStream_t st) {
  if (inst)
    launch_life_c<R, ADJ, true>(P, nblk, st);
  else
    launch_life_c<R, ADJ, false>(P, nblk, st);
  HIPCHK(hipGetLastError());
  return 0;
}

// Events per package kept in the adjoint's event scratch (more are walked
// again in pass B), and the sizes of that scratch and of the peel-ray queue
// that bound a chunk of packages (each at most a quarter of the free device
// memory).  Every chunk costs its launches' tails (a persistent kernel ends
// with few waves busy), so the budgets are large: the 1e7-package spiral
// runs in one chunk of each.  A larger chunk also puts more rays into each
// pixel's run of the sorted queue, where the peel walks share more cells,
// but spreads the jobs that the walks read in sorted order over a larger
// array: the clumpy 512^3 forward (1e8 packages) takes 1920 / 1829 / 1799 /
// 1786 ms with a queue of 8 / 16 / 24 / 32 GiB (14 / 7 / 5 / 4 chunks; peel
// walks 482 / 422 / 401 / 391 ms), and 1829 / 1863 ms in 3 / 2 chunks (peel
// walks 444 / 496 ms).
constexpr int kEventsKept = 32;
constexpr size_t kScratchBytes = size_t(1) << 34, kQueueBytes = size_t(1) << 35;

// Shared driver of run_photons and backward_density.
int life(bool adjoint, const mcrt_grid* grid, const void* rho_dev, const mcrt_optics* optics, int n_src,
         const mcrt_source* sources, int n_det, const mcrt_detector* detectors, const mcrt_opts* opts,
         double* images_dev, double* absorbed_dev, const double* adj_dev, const double* adj_abs_dev,
         const mcrt_grads* grads, mcrt_stats* stats, void* hip_stream) {
  host::Prepared pr;
  if (int e = host::prepare(grid, rho_dev, optics, n_src, sources, n_det, detectors, opts, pr)) return e;
  RunParams& P = pr.P;
  const bool peel = (opts->flags & (MCRT_PEEL_EMIT | MCRT_PEEL_SCAT)) && n_det > 0;
  if (!adjoint) {
    if (peel && !images_dev) return fail(MCRT_EINVAL, "images_dev is NULL");
    if ((opts->flags & MCRT_ABSORB) && !absorbed_dev) return fail(MCRT_EINVAL, "absorbed_dev is NULL with MCRT_ABSORB");
    P.images = images_dev;
    P.absorbed = (opts->flags & MCRT_ABSORB) ? absorbed_dev : nullptr;
  } else {
    if (peel && !adj_dev) return fail(MCRT_EINVAL, "adj_images_dev is NULL");
    if (!grads) return fail(MCRT_EINVAL, "grads is NULL");
    if (!grads->rho && !grads->albedo && !grads->g && !grads->lum) return fail(MCRT_EINVAL, "no gradient requested");
    P.adj = adj_dev;
    P.grad = grads->rho;
  }
  // the attached gradient: densities of an image loss, frames and SED
  // instruments, a workspace of every event of a package
  const bool att = adjoint && (opts->flags & MCRT_ATTACHED);
  int att_ev = 0;
  if (att)
    if (int e = host::attached_check(*optics, n_det, detectors, *opts, adj_abs_dev != nullptr,
                                     grads->albedo || grads->g || grads->lum || !grads->rho, &att_ev))
      return e;
  const int nl = P.n_lambda;
  const bool f32 = opts->precision == MCRT_PREC_FP32;
  int nblk = 0;
  const int kind = P.G.kind;
  bool inst = false;  // instruments other than frames (SED, camera)
  for (int d = 0; d < n_det; ++d) inst = inst || pr.det[d].kind != kDetFrame;
  const bool optg = adjoint && (grads->albedo || grads->g || grads->lum);
  // the life kernels' full variant also carries the optics and absorbed-tally gradients
  const bool full = inst || optg || (adjoint && adj_abs_dev);
  if (int e = adjoint ? (f32 ? life_grid<float, true>(kind, full, opts->launch_blocks, &nblk)
                             : life_grid<double, true>(kind, full, opts->launch_blocks, &nblk))
                      : (f32 ? life_grid<float, false>(kind, full, opts->launch_blocks, &nblk)
                             : life_grid<double, false>(kind, full, opts->launch_blocks, &nblk)))
    return e;
  // the adjoint tape (mcrt_opts.tape): the forward run writes it; an
  // adjoint with a usable tape fills its event scratch from it and replays
  // each package once
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const uint64_t tape_need = peel ? host::tape_bytes(optics, n_det, opts) : 0;
  const int tape_ev = tape_need ? (int)host::tape_events(*optics, *opts) : 0;
  bool tape_fwd = false, tape_adj = false;
  uint64_t fprint = 0;
  if (opts->tape && !att) {
    if (!tape_need) return fail(MCRT_EINVAL, "tape given, but this run cannot keep one (mcrt_tape_bytes is 0)");
    fprint = host::tape_fingerprint(*grid, *optics, n_src, sources, n_det, detectors, *opts);
    if (!adjoint) {
      if (opts->tape_bytes < tape_need)
        return fail(MCRT_EINVAL, "tape_bytes %llu < %llu", (unsigned long long)opts->tape_bytes,
                    (unsigned long long)tape_need);
      tape_fwd = true;
    } else {
      host::TapeHeader hdr;
      HIPCHK(hipMemcpyAsync(&hdr, opts->tape, sizeof hdr, hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      bool usable = false;
      if (int e = host::check_tape(hdr, fprint, P.n_items, tape_ev, n_det, opts->tape_bytes, tape_need, &usable))
        return e;
      tape_adj = usable && !adj_abs_dev;
    }
  }
  const unsigned char* const tape_base = static_cast<const unsigned char*>(opts->tape);
  const size_t tape_pix_off = host::kTapeHeader + align256(sizeof(double) * (size_t)P.n_items * tape_ev * (1 + n_det));
  // packages run in equal chunks: the adjoint's event scratch holds, per
  // package, T and q per frame for ev_max events (the tape's events, else
  // kEventsKept) plus the sum of q beyond; the peel-ray queue by default 8
  // rays per package and frame
  // (the attached gradient: kAttF doubles for each of a package's events)
  const int ev_max = att ? att_ev : (tape_adj ? tape_ev : kEventsKept);
  const int ev_k = att ? (int)kAttF : 1 + n_det + (adjoint && adj_abs_dev ? 1 : 0);  // T, q per frame, then B of the path
  const size_t per_item = sizeof(double) * ((size_t)ev_max * ev_k + (att ? 0 : 1 + (optg ? 4 : 0)));
  const bool queued = peel && opts->peel_queue != -1;  // the attached gradient queues its deposit walks only
  P.depth_drop = adjoint ? kDepthDropAdjoint : 0;
  size_t free_b = 0, total_b = 0;
  HIPCHK(hipMemGetInfo(&free_b, &total_b));
  unsigned long long most = P.n_items;
  if (adjoint)
    most = std::min<unsigned long long>(most, std::max<size_t>(1 << 16, std::min(kScratchBytes, free_b / 4) / per_item));
  if (queued && opts->peel_queue == 0)
    most = std::min<unsigned long long>(
        most, std::max<size_t>(1 << 16, std::min(kQueueBytes, free_b / 4) /
                                            ((size_t)n_det * 8 * kQueueBytesPerRay)));
  if (opts->max_chunk > 0) most = std::min<unsigned long long>(most, (unsigned long long)opts->max_chunk);
  const unsigned long long n_chunks = (P.n_items + most - 1) / most;
  const unsigned long long chunk = (P.n_items + n_chunks - 1) / n_chunks;
  // the adjoint's event scratch, then (optics gradients) the pass-B sums
  const size_t n_evs = adjoint ? (size_t)chunk * ((size_t)ev_max * ev_k + (att ? 0 : 1 + (optg ? 4 : 0))) : 0;
  const long long n_tally = adjoint ? (long long)P.G.ncell_pad : (P.absorbed ? (long long)nl * P.G.ntal : 0);
  const size_t off_lam = 0;
  const size_t off_det = align256(sizeof(LamDev) * nl);
  const size_t off_src = off_det + align256(sizeof(DetDev) * pr.det.size());
  const size_t off_pl = off_src + align256(sizeof(SrcDev) * pr.src.size());
  const size_t off_cnt = off_pl + host::plane_bytes(P.G, *grid);
  const size_t off_rho = off_cnt + 256;
  const size_t off_tal = off_rho + align256((size_t)P.G.ncell_pad * (f32 ? 4 : 8));
  const size_t off_evs = off_tal + align256(sizeof(double) * (size_t)n_tally);
  // a cell source: its CDF [n_lambda][ncell + 1], the scan's tile sums, the
  // per-wavelength totals and a flag for bad luminosities
  const bool cells = pr.cell_src >= 0;
  const long long cdf_tiles = cells ? ((long long)P.G.ncell + kCdfTile - 1) / kCdfTile : 0;
  if (cells && (long long)nl * cdf_tiles * kCdfThreads >= (1ll << 32))
    return fail(MCRT_EINVAL, "cell source: n_lambda x cells too large");
  const size_t off_cum = off_evs + align256(sizeof(double) * n_evs);
  const size_t off_cts = off_cum + align256(cells ? sizeof(double) * (size_t)nl * (P.G.ncell + 1) : 0);
  const size_t off_ctot = off_cts + align256(sizeof(double) * (size_t)(nl * cdf_tiles));
  const size_t off_lums = off_ctot + (cells ? align256(sizeof(double) * nl + 8) : 0);
  const size_t off_aab = off_lums + (optg ? align256(sizeof(double) * pr.lums.size()) : 0);
  const bool aabs = adjoint && adj_abs_dev;  // a loss on the absorbed tally: its adjoint, bricked
  const size_t bytes = off_aab + (aabs ? align256(sizeof(double) * (size_t)nl * P.G.ncell_pad) : 0);

  DeviceBlock blk;
  blk.st = st;
  HIPCHK(hipMallocAsync(reinterpret_cast<void**>(&blk.ptr), bytes, st));
  if (cells) {
    double* cum = reinterpret_cast<double*>(blk.ptr + off_cum);
    if (int e = cell_cdf(static_cast<const double*>(sources[pr.cell_src].cell_lum), nl, P.G.ncell, cum,
                         reinterpret_cast<double*>(blk.ptr + off_cts), (int)cdf_tiles,
                         reinterpret_cast<double*>(blk.ptr + off_ctot), st, &pr, n_src, sources, opts))
      return e;
    pr.src[pr.cell_src].cum = cum;
  }
  std::vector<unsigned char> blob(off_rho, 0);
  std::memcpy(blob.data() + off_lam, pr.lam.data(), sizeof(LamDev) * nl);
  std::memcpy(blob.data() + off_det, pr.det.data(), sizeof(DetDev) * pr.det.size());
  std::memcpy(blob.data() + off_src, pr.src.data(), sizeof(SrcDev) * pr.src.size());
  host::put_planes(*grid, P.G, blob.data() + off_pl, blk.ptr + off_pl);
  HIPCHK(hipMemcpyAsync(blk.ptr, blob.data(), off_rho, hipMemcpyHostToDevice, st));
  if (int e = brick_density(P.G, rho_dev, blk.ptr + off_rho, f32, st)) return e;
  double* const user_tally = adjoint ? P.grad : P.absorbed;
  double* const tally = n_tally ? reinterpret_cast<double*>(blk.ptr + off_tal) : nullptr;
  P.rho = blk.ptr + off_rho;
  if (adjoint)
    P.grad = tally;
  else
    P.absorbed = tally;
  if (adjoint) {
    P.evs = reinterpret_cast<double*>(blk.ptr + off_evs);
    P.ev_max = ev_max;
    P.ev_k = ev_k;
  }
  if (tape_fwd) {  // header with the run's fingerprint, then every T, C and image index 0
    unsigned char* t = static_cast<unsigned char*>(opts->tape);
    const host::TapeHeader hdr = host::tape_header(fprint, P.n_items, tape_ev, n_det);
    HIPCHK(hipMemcpyAsync(t, &hdr, sizeof hdr, hipMemcpyHostToDevice, st));
    const long long words = (long long)((tape_need - host::kTapeHeader) / 4);
    hipLaunchKernelGGL(k_zero_u32, dim3(stream_blocks(words)), dim3(kBlock), 0, st,
                       reinterpret_cast<unsigned*>(t + host::kTapeHeader), words);
    HIPCHK(hipGetLastError());
    P.tape = reinterpret_cast<double*>(t + host::kTapeHeader);
    P.tape_pix = reinterpret_cast<unsigned*>(t + tape_pix_off);
    P.tape_over = reinterpret_cast<unsigned*>(t + offsetof(host::TapeHeader, overflow));
    P.tape_ev = tape_ev;
    P.tape_n = P.n_items;
  }
  double* const lums = optg ? reinterpret_cast<double*>(blk.ptr + off_lums) : nullptr;
  if (aabs) {
    double* aab = reinterpret_cast<double*>(blk.ptr + off_aab);
    for (int l = 0; l < nl; ++l)
      if (int e = brick_density(P.G, adj_abs_dev + (size_t)l * P.G.ncell, aab + (size_t)l * P.G.ncell_pad, false, st))
        return e;
    P.adj_abs = aab;
  }
  if (optg) {  // the sources' luminosities (known once the cell CDF is); gradients start at 0
    HIPCHK(hipMemcpyAsync(lums, pr.lums.data(), sizeof(double) * pr.lums.size(), hipMemcpyHostToDevice, st));
    if (int e = zero_fill(grads->albedo, grads->albedo ? nl : 0, st)) return e;
    if (int e = zero_fill(grads->g, grads->g ? nl : 0, st)) return e;
    if (int e = zero_fill(grads->lum, grads->lum ? (long long)n_src * nl : 0, st)) return e;
  }
  P.item0 = 0;
  P.n_chunk = P.n_items;
  P.lam = reinterpret_cast<const LamDev*>(blk.ptr + off_lam);
  P.det = reinterpret_cast<const DetDev*>(blk.ptr + off_det);
  P.src = reinterpret_cast<const SrcDev*>(blk.ptr + off_src);
  P.work = reinterpret_cast<unsigned long long*>(blk.ptr + off_cnt);
  P.dstats = reinterpret_cast<double*>(blk.ptr + off_cnt + 64);
  P.xstats = reinterpret_cast<unsigned long long*>(blk.ptr + off_cnt + 128);
  if (!adjoint)
    if (int e = zero_fill(P.images, peel ? pr.n_images : 0, st)) return e;
  if (int e = zero_fill(tally, n_tally, st)) return e;
  PeelQueue queue;
  if (queued) {
    if (int e = make_peel_queue(*opts, pr, chunk, st, queue)) return e;
    P.jobs = queue.cap ? queue.jobs : nullptr;
    P.keys = queue.cap ? queue.keys : nullptr;
    P.job_cap = queue.cap;
  }
  unsigned long long* const ctr = reinterpret_cast<unsigned long long*>(blk.ptr + off_cnt);
  EventPair ev;
  Spans sp;
  sp.on = stats != nullptr;
  if (stats) {
    HIPCHK(hipEventCreate(&ev.a));
    HIPCHK(hipEventCreate(&ev.c));
    HIPCHK(hipEventRecord(ev.a, st));
  }
  unsigned long long launches = 0;  // of the life-cycle kernel
  auto queue_phase = [&](bool adj) -> int {  // sort and walk the chunk's queued peel rays
    return adj ? (f32 ? run_peel_jobs<float, true>(queue, P, ctr, inst, st, sp)
                      : run_peel_jobs<double, true>(queue, P, ctr, inst, st, sp))
               : (f32 ? run_peel_jobs<float, false>(queue, P, ctr, inst, st, sp)
                      : run_peel_jobs<double, false>(queue, P, ctr, inst, st, sp));
  };
  auto life_launch = [&](bool adj) -> int {
    if (int e = sp.mark(kSpanLife, st)) return e;
    const int r = adj ? (f32 ? launch_life<float, true>(P, full, nblk, st) : launch_life<double, true>(P, full, nblk, st))
                      : (f32 ? launch_life<float, false>(P, full, nblk, st)
                             : launch_life<double, false>(P, full, nblk, st));
    if (r) return r;
    ++launches;
    return sp.mark(kSpanLife, st);
  };
  if (!adjoint) {
    for (unsigned long long c0 = 0; c0 < P.n_items; c0 += chunk) {
      P.item0 = c0;
      P.n_chunk = std::min(chunk, P.n_items - c0);
      if (int e = reset_counters(ctr, 0, 1, st)) return e;
      if (int e = reset_counters(ctr, kJobCounter, 2, st)) return e;
      if (int e = life_launch(false)) return e;
      if (P.jobs)
        if (int e = queue_phase(false)) return e;
    }
  } else if (att) {
    if (int e = reset_counters(ctr, kAttOverflow, 2, st)) return e;
    for (unsigned long long c0 = 0; c0 < P.n_items; c0 += chunk) {
      P.item0 = c0;
      P.n_chunk = std::min(chunk, P.n_items - c0);
      if (int e = reset_counters(ctr, 0, 1, st)) return e;
      if (int e = reset_counters(ctr, kJobCounter, 2, st)) return e;
      if (int e = reset_counters(ctr, kDepCounter, 1, st)) return e;
      P.dep_jobs = 1;  // the queued rays carry their weights
      if (int e = sp.mark(kSpanLife, st)) return e;
      if (int e = launch_attached(P, f32, st)) return e;
      ++launches;
      if (int e = sp.mark(kSpanLife, st)) return e;
      // the queued deposit walks, in FP64 like the sweeps' own walks
      if (P.jobs)
        if (int e = run_peel_jobs<double, true>(queue, P, ctr, inst, st, sp)) return e;
    }
  } else {
    for (unsigned long long c0 = 0; c0 < P.n_items; c0 += chunk) {
      P.item0 = c0;
      P.n_chunk = std::min(chunk, P.n_items - c0);
      P.gpart = optg ? P.evs + P.n_chunk * ((unsigned long long)ev_max * ev_k + 1) : nullptr;
      if (tape_adj) {  // the scratch from the tape, then pass B alone, then the deposit walks
        if (int e = zero_fill(P.gpart, optg ? 4 * (long long)P.n_chunk : 0, st)) return e;
        hipLaunchKernelGGL(k_tape_q, dim3(stream_blocks((long long)P.n_chunk)), dim3(kBlock), 0, st,
                           reinterpret_cast<const double*>(tape_base + host::kTapeHeader),
                           reinterpret_cast<const unsigned*>(tape_base + tape_pix_off), P.adj, P.evs, P.item0,
                           P.n_chunk, (unsigned long long)P.n_items, ev_max, n_det);
        HIPCHK(hipGetLastError());
        if (int e = reset_counters(ctr, 0, 1, st)) return e;
        if (int e = reset_counters(ctr, kJobCounter, 2, st)) return e;
        if (int e = reset_counters(ctr, kDepCounter, 1, st)) return e;
        P.split = 2;
        P.dep_jobs = 1;
        if (opts->event_batch == 0) P.batch = kBatchPassB;
        if (int e = life_launch(true)) return e;
        if (P.jobs)
          if (int e = queue_phase(true)) return e;
      } else {  // pass A, the queue's walks, pass B
        const long long n_scr = (long long)(P.n_chunk * ((unsigned long long)ev_max * ev_k + 1 + (optg ? 4 : 0)));
        if (int e = zero_fill(P.evs, n_scr, st)) return e;
        if (int e = reset_counters(ctr, 0, 1, st)) return e;
        if (int e = reset_counters(ctr, kJobCounter, 2, st)) return e;
        if (int e = reset_counters(ctr, kDepCounter, 1, st)) return e;
        P.split = 1;  // pass A
        if (opts->event_batch == 0) P.batch = kBatchPassA;
        if (int e = life_launch(true)) return e;
        if (P.jobs)
          if (int e = queue_phase(true)) return e;
        if (int e = reset_counters(ctr, 0, 1, st)) return e;
        P.split = 2;  // pass B
        if (opts->event_batch == 0) P.batch = kBatchPassB;
        if (int e = life_launch(true)) return e;
      }
      if (optg) {
        const unsigned nb = (unsigned)((P.item0 + P.n_chunk - 1) / P.n_pkg - P.item0 / P.n_pkg + 1);
        hipLaunchKernelGGL(k_grad_optics, dim3(nb), dim3(kOptThreads), 0, st, P.gpart, P.item0, P.n_chunk, P.n_pkg,
                           n_src, P.lam, lums, nl, grads->albedo, grads->g, grads->lum);
        HIPCHK(hipGetLastError());
      }
    }
  }
  if (stats) HIPCHK(hipEventRecord(ev.c, st));
  if (tally && user_tally)
    if (int e = unbrick_tally(P.G, tally, user_tally, adjoint ? 1 : nl, !adjoint, st)) return e;
  if (att) {  // a package beyond the event bound (not expected: the bound holds by construction)
    unsigned long long over = 0;
    HIPCHK(hipMemcpyAsync(&over, ctr + kAttOverflow, sizeof over, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (over) return fail(MCRT_EOVERFLOW, "MCRT_ATTACHED: a package had more events than %d", att_ev);
  }
  if (stats) {
    double ds[3];
    unsigned long long xs[7], xq[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(ds, P.dstats, sizeof ds, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(xs, P.xstats, sizeof xs, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(xq, ctr + kQueueCrossings, sizeof xq, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, ev.a, ev.c) != hipSuccess) ms = -1.0f;
    const double ms_sort = sp.ms(kSpanSort), ms_peel = sp.ms(kSpanPeel), ms_dep = sp.ms(kSpanDep);
    stats->emitted = pr.emitted;
    stats->absorbed = ds[0];
    stats->escaped = ds[1];
    stats->truncated = ds[2];
    stats->x_path = xs[0];
    stats->x_locate = xs[1];
    stats->x_peel = xs[2] + xq[0];
    stats->events = xs[3];
    stats->packages = xs[4];
    stats->peels = xs[5];
    stats->deposits = xs[6] + xq[1];
    stats->kernel_ms = ms;
    stats->x_queue = xq[0];
    stats->life_ms = sp.ms(kSpanLife);
    stats->queue_ms = ms_sort + ms_peel + ms_dep;
    stats->sort_ms = ms_sort;
    stats->peel_ms = ms_peel;
    stats->dep_ms = ms_dep;
    stats->d_queue = xq[1];
    if (att) {  // the crossings of the peel rays' deposit walks: those the attached kernel walked, then the queue's
      uint64_t inline_dep = 0;
      HIPCHK(hipMemcpyAsync(&inline_dep, ctr + kAttDepCrossings, sizeof(uint64_t), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      stats->d_queue = inline_dep + xq[1];
    }
    stats->life_launches = launches;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// trace_path and its variant that allocates nothing.
//
// The variant's device block (counters, plane or tree tables, bricked
// densities) is `scratch` (above), a file-scope device array: every device
// holds its own copy at its own address, taken once per device with
// hipGetSymbolAddress (in host code the array's name is not a device
// address).  Calls on one device share it and must not overlap.

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// The current device's address of `scratch` (set up on its first use).
int scratch_address(unsigned char** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MCRT_EINVAL, "device %d beyond the %d the library tracks", dev,
                                                 kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(MCRT_EHIP, "hipGetSymbolAddress gave no address for the scratch array");
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return 0;
}

// trace_path's work.  fixed = false: the device block is allocated on the
// stream and freed there when the work ends; fixed = true: it is the
// scratch array (sizes beyond it are rejected before any device work), and
// the counters are cleared by a fill kernel rather than by the copy of the
// tables, which only rectilinear and tree grids need.
int trace_impl(const mcrt_grid* grid, const void* rho_dev, double kappa, int precision, int64_t n_rays,
               const double* origin_dev, const double* dir_dev, double* tau_dev, int32_t max_seg,
               int32_t* seg_cell_dev, double* seg_len_dev, int32_t* n_seg_dev, uint64_t* crossings_host,
               void* hip_stream, bool fixed) {
  if (int e = host::check_trace(grid, rho_dev, kappa, precision, n_rays, origin_dev, dir_dev, tau_dev, max_seg,
                                seg_cell_dev, seg_len_dev))
    return e;
  const bool lists = seg_cell_dev != nullptr;
  TraceParams P;
  std::memset(&P, 0, sizeof P);
  if (int e = host::make_grid(*grid, host::elem_bytes(precision), 0, P.G)) return e;
  const bool f32 = precision == MCRT_PREC_FP32;
  const size_t tables = host::plane_bytes(P.G, *grid);
  const size_t off_rho = 256 + tables;  // counters, plane tables, densities
  const size_t bytes = off_rho + (size_t)P.G.ncell_pad * (f32 ? 4 : 8);
  if (fixed && bytes > (size_t)MCRT_NOALLOC_SCRATCH_BYTES)
    return fail(MCRT_EINVAL, "trace_path_noalloc: the grid needs %zu bytes of device scratch, the limit is %zu", bytes,
                (size_t)MCRT_NOALLOC_SCRATCH_BYTES);
  if (n_rays == 0) {
    if (crossings_host) *crossings_host = 0;
    return 0;
  }
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  P.kappa = kappa;
  P.n_rays = n_rays;
  P.origin = origin_dev;
  P.dir = dir_dev;
  P.tau = tau_dev;
  P.max_seg = lists ? max_seg : 0;
  P.seg_cell = lists ? seg_cell_dev : nullptr;
  P.seg_len = lists ? seg_len_dev : nullptr;
  P.n_seg = n_seg_dev;
  P.batch = kBatchQueue;
  DeviceBlock blk;  // frees only what it allocated
  blk.st = st;
  unsigned char* base = nullptr;
  if (fixed) {
    if (int e = scratch_address(&base)) return e;
  } else {
    HIPCHK(hipMallocAsync(reinterpret_cast<void**>(&blk.ptr), bytes, st));
    base = blk.ptr;
  }
  if (tables || !fixed) {
    std::vector<unsigned char> blob(off_rho, 0);
    host::put_planes(*grid, P.G, blob.data() + 256, base + 256);
    HIPCHK(hipMemcpyAsync(base, blob.data(), off_rho, hipMemcpyHostToDevice, st));
  }
  if (fixed) hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, st, reinterpret_cast<unsigned*>(base), 64ll);
  if (int e = brick_density(P.G, rho_dev, base + off_rho, f32, st)) return e;
  P.rho = base + off_rho;
  P.work = reinterpret_cast<unsigned long long*>(base);
  P.counters = P.work + 1;
  const int r = f32 ? launch_by_kind<TraceParams, float>(P, st, k_trace<float, kGridRegular>,
                                                         k_trace<float, kGridRect>, k_trace<float, kGridTree>,
                                                         kTraceBlocksPerCu)
                    : launch_by_kind<TraceParams, double>(P, st, k_trace<double, kGridRegular>,
                                                          k_trace<double, kGridRect>, k_trace<double, kGridTree>,
                                                          kTraceBlocksPerCu);
  if (r) return r;
  HIPCHK(hipGetLastError());
  if (crossings_host || lists) {
    unsigned long long c[2] = {0, 0};
    HIPCHK(hipMemcpyAsync(c, P.counters, sizeof c, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if (crossings_host) *crossings_host = c[0];
    if (lists && c[1]) return fail(MCRT_EOVERFLOW, "%llu rays had more than max_seg = %d segments", c[1], max_seg);
  }
  return 0;
}

}  // namespace

extern "C" {

int mcrt_abi_version(void) { return MCRT_ABI_VERSION; }

uint64_t mcrt_tape_bytes(const mcrt_optics* optics, int n_det, const mcrt_opts* opts) {
  try {
    return mcrt::host::tape_bytes(optics, n_det, opts);
  } catch (...) {
    return 0;
  }
}

const char* mcrt_last_error(void) { return mcrt::host::last_error().c_str(); }

int run_photons(const mcrt_grid* grid, const void* rho_dev, const mcrt_optics* optics, int n_src,
                const mcrt_source* sources, int n_det, const mcrt_detector* detectors, const mcrt_opts* opts,
                double* images_dev, double* absorbed_dev, mcrt_stats* stats_host, void* hip_stream) {
  try {
    mcrt::host::last_error().clear();
    return life(false, grid, rho_dev, optics, n_src, sources, n_det, detectors, opts, images_dev, absorbed_dev,
                nullptr, nullptr, nullptr, stats_host, hip_stream);
  } catch (...) {
    return fail(MCRT_EHIP, "run_photons: host exception");
  }
}

int backward_density(const mcrt_grid* grid, const void* rho_dev, const mcrt_optics* optics, int n_src,
                     const mcrt_source* sources, int n_det, const mcrt_detector* detectors, const mcrt_opts* opts,
                     const double* adj_images_dev, double* grad_rho_dev, mcrt_stats* stats_host,
                     void* hip_stream) {
  try {
    mcrt::host::last_error().clear();
    mcrt_opts o;
    if (opts) {
      o = *opts;
      o.flags &= ~MCRT_ABSORB;
    }
    mcrt_grads g = {grad_rho_dev, nullptr, nullptr, nullptr};
    if (!grad_rho_dev) return fail(MCRT_EINVAL, "grad_rho_dev is NULL");
    return life(true, grid, rho_dev, optics, n_src, sources, n_det, detectors, opts ? &o : nullptr, nullptr,
                nullptr, adj_images_dev, nullptr, &g, stats_host, hip_stream);
  } catch (...) {
    return fail(MCRT_EHIP, "backward_density: host exception");
  }
}

int backward(const mcrt_grid* grid, const void* rho_dev, const mcrt_optics* optics, int n_src,
             const mcrt_source* sources, int n_det, const mcrt_detector* detectors, const mcrt_opts* opts,
             const double* adj_images_dev, const double* adj_absorbed_dev, const mcrt_grads* grads,
             mcrt_stats* stats_host, void* hip_stream) {
  try {
    mcrt::host::last_error().clear();
    mcrt_opts o;
    if (opts) {
      o = *opts;
      o.flags &= ~MCRT_ABSORB;
    }
    if (adj_absorbed_dev && grads && !grads->rho)
      return fail(MCRT_EINVAL, "adj_absorbed_dev needs grads->rho (its optics gradients are not computed)");
    return life(true, grid, rho_dev, optics, n_src, sources, n_det, detectors, opts ? &o : nullptr, nullptr,
                nullptr, adj_images_dev, adj_absorbed_dev, grads, stats_host, hip_stream);
  } catch (...) {
    return fail(MCRT_EHIP, "backward: host exception");
  }
}

int trace_path(const mcrt_grid* grid, const void* rho_dev, double kappa, int precision, int64_t n_rays,
               const double* origin_dev, const double* dir_dev, double* tau_dev, int32_t max_seg,
               int32_t* seg_cell_dev, double* seg_len_dev, int32_t* n_seg_dev, uint64_t* crossings_host,
               void* hip_stream) {
  try {
    mcrt::host::last_error().clear();
    return trace_impl(grid, rho_dev, kappa, precision, n_rays, origin_dev, dir_dev, tau_dev, max_seg, seg_cell_dev,
                      seg_len_dev, n_seg_dev, crossings_host, hip_stream, false);
  } catch (...) {
    return fail(MCRT_EHIP, "trace_path: host exception");
  }
}

int trace_path_noalloc(const mcrt_grid* grid, const void* rho_dev, double kappa, int precision, int64_t n_rays,
                       const double* origin_dev, const double* dir_dev, double* tau_dev, int32_t max_seg,
                       int32_t* seg_cell_dev, double* seg_len_dev, int32_t* n_seg_dev, uint64_t* crossings_host,
                       void* hip_stream) {
  try {
    mcrt::host::last_error().clear();
    return trace_impl(grid, rho_dev, kappa, precision, n_rays, origin_dev, dir_dev, tau_dev, max_seg, seg_cell_dev,
                      seg_len_dev, n_seg_dev, crossings_host, hip_stream, true);
  } catch (...) {
    return fail(MCRT_EHIP, "trace_path_noalloc: host exception");
  }
}

int peel_off(const mcrt_grid* grid, const void* rho_dev, double kappa, double g, int precision, int64_t n_events,
             const double* pos_dev, const double* dir_in_dev, const double* w_dev, int n_det,
             const mcrt_detector* detectors, double* images_dev, void* hip_stream) {
  try {
    mcrt::host::last_error().clear();
    if (int e = host::check_peel(grid, rho_dev, kappa, g, precision, n_events, pos_dev, w_dev, n_det, detectors,
                                 images_dev))
      return e;
    if (n_events == 0) return 0;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    PeelParams P;
    std::memset(&P, 0, sizeof P);
    if (int e = host::make_grid(*grid, host::elem_bytes(precision), 0, P.G)) return e;
    const bool f32 = precision == MCRT_PREC_FP32;
    std::vector<DetDev> det = host::make_dets(n_det, detectors, nullptr);
    const size_t off_cnt = align256(sizeof(DetDev) * det.size());
    const size_t off_pl = off_cnt + 256;
    const size_t off_rho = off_pl + host::plane_bytes(P.G, *grid);
    const size_t bytes = off_rho + (size_t)P.G.ncell_pad * (f32 ? 4 : 8);
    std::vector<unsigned char> blob(off_rho, 0);
    std::memcpy(blob.data(), det.data(), sizeof(DetDev) * det.size());
    DeviceBlock blk;
    blk.st = st;
    HIPCHK(hipMallocAsync(reinterpret_cast<void**>(&blk.ptr), bytes, st));
    host::put_planes(*grid, P.G, blob.data() + off_pl, blk.ptr + off_pl);
    HIPCHK(hipMemcpyAsync(blk.ptr, blob.data(), off_rho, hipMemcpyHostToDevice, st));
    if (int e = brick_density(P.G, rho_dev, blk.ptr + off_rho, f32, st)) return e;
    P.rho = blk.ptr + off_rho;
    P.kappa = kappa;
    P.g = g;
    P.n_events = n_events;
    P.n_det = n_det;
    P.det = reinterpret_cast<const DetDev*>(blk.ptr);
    P.pos = pos_dev;
    P.dir_in = dir_in_dev;
    P.w = w_dev;
    P.images = images_dev;
    P.work = reinterpret_cast<unsigned long long*>(blk.ptr + off_cnt);
    P.batch = kBatchQueue;
    const int r = f32 ? launch_by_kind<PeelParams, float>(P, st, k_peel<float, kGridRegular>,
                                                          k_peel<float, kGridRect>, k_peel<float, kGridTree>)
                      : launch_by_kind<PeelParams, double>(P, st, k_peel<double, kGridRegular>,
                                                           k_peel<double, kGridRect>, k_peel<double, kGridTree>);
    if (r) return r;
    HIPCHK(hipGetLastError());
    return 0;
  } catch (...) {
    return fail(MCRT_EHIP, "peel_off: host exception");
  }
}

int dust_emission(const mcrt_grid* grid, const void* rho_dev, int precision, int n_abs, const double* absorbed_dev,
                  int n_lambda, const double* lambda, const double* dlambda, const double* kappa_abs,
                  double emissivity, double* temperature_dev, double* emission_dev, void* hip_stream) {
  try {
    mcrt::host::last_error().clear();
    if (int e = host::check_dust(grid, rho_dev, precision, n_abs, absorbed_dev, n_lambda, lambda, dlambda, kappa_abs,
                                 emissivity, emission_dev))
      return e;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    DustParams P;
    std::memset(&P, 0, sizeof P);
    if (int e = host::make_grid(*grid, host::elem_bytes(precision), 0, P.G)) return e;
    // plane or tree tables, a, b, the ln P table
    const size_t off_a = host::plane_bytes(P.G, *grid), off_b = off_a + align256(sizeof(double) * n_lambda),
                 off_t = off_b + align256(sizeof(double) * n_lambda),
                 bytes = off_t + align256(sizeof(double) * (kDustTable + 1));
    std::vector<unsigned char> blob(off_t, 0);
    DeviceBlock blk;
    blk.st = st;
    HIPCHK(hipMallocAsync(reinterpret_cast<void**>(&blk.ptr), bytes, st));
    host::put_planes(*grid, P.G, blob.data(), blk.ptr);
    host::dust_constants(n_lambda, lambda, dlambda, kappa_abs, reinterpret_cast<double*>(blob.data() + off_a),
                         reinterpret_cast<double*>(blob.data() + off_b));
    HIPCHK(hipMemcpyAsync(blk.ptr, blob.data(), off_t, hipMemcpyHostToDevice, st));
    P.D.nl = n_lambda;
    P.D.a = reinterpret_cast<const double*>(blk.ptr + off_a);
    P.D.b = reinterpret_cast<const double*>(blk.ptr + off_b);
    P.D.lnP = reinterpret_cast<const double*>(blk.ptr + off_t);
    hipLaunchKernelGGL(k_dust_table, dim3((kDustTable + 256) / 256), dim3(256), 0, st, P.D,
                       reinterpret_cast<double*>(blk.ptr + off_t));
    P.rho = rho_dev;
    P.absorbed = absorbed_dev;
    P.n_abs = n_abs;
    P.emissivity = emissivity;
    P.temperature = temperature_dev;
    P.emission = emission_dev;
    const dim3 g((unsigned)((P.G.ncell + kBlock - 1) / kBlock)), b(kBlock);
    const bool f32 = precision == MCRT_PREC_FP32;
    const int kind = P.G.kind;
    void (*kern)(DustParams) =
        f32 ? (kind == kGridRect   ? k_dust_emission<float, kGridRect>
               : kind == kGridTree ? k_dust_emission<float, kGridTree>
                                   : k_dust_emission<float, kGridRegular>)
            : (kind == kGridRect   ? k_dust_emission<double, kGridRect>
               : kind == kGridTree ? k_dust_emission<double, kGridTree>
                                   : k_dust_emission<double, kGridRegular>);
    hipLaunchKernelGGL(kern, g, b, 0, st, P);
    HIPCHK(hipGetLastError());
    return 0;
  } catch (...) {
    return fail(MCRT_EHIP, "dust_emission: host exception");
  }
}

}  // extern "C"
