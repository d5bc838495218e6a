// libpdyn: C-ABI entry points and HIP kernels for gfx950.
//
// Kernel map (one lane = one state; consecutive lanes = consecutive states):
//   k_link_table       per link: the derived 32-word record (rotation of M_i
//                      from its quaternion, twist norms, h = m c, I_O) -- a map.
//   k_link_table_ilv   the same records for one chain per state, interleaved
//                      over the lanes of each wavefront.
//   k_dynamics         per state: the sweeps of sweeps.hpp (ID, FD or both).
//   k_dynamics_split   per 64 states, 3-5 wavefronts with LDS hand-offs: the
//                      transform producers, the articulated-inertia pass, the
//                      bias passes and (ID+FD) the inverse dynamics.
//   k_id_split         per 64 states, 2 wavefronts: transforms, Newton-Euler.
//   k_vjp              per state: the adjoint sweeps (ID or FD vector-Jacobian
//                      product), inertia cotangents summed per wave.
//   k_vjp_split        per 64 states, 2-4 wavefronts: the adjoints cut into
//                      passes (cotangent / solve, Newton-Euler, articulated
//                      inertia, adjoint recursion, outputs) with LDS hand-offs.
//   k_reduce_lanes     per (link, parameter): sum over states of the per-lane
//                      inertia cotangents (fixed order).
//   k_rollout          per state: T steps of forward dynamics + semi-implicit
//                      Euler in one launch, (q, qd) checkpoints every k steps.
//   k_rollout_vjp      per state: the rollout adjoint, segment by segment from
//                      the checkpoints (recompute k steps, then k reverse steps).
//   k_id_team          per chain, P lanes: inverse dynamics by segmented scans.
//   k_jsiia            per state: M(q) by composite bodies, and forward
//                      dynamics by its Cholesky factorisation (jsiia.hpp).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pdyn.h"
#include "abi_scan.hpp"
#include "fd_scan.hpp"
#include "hessian.hpp"
#include "jsiia.hpp"
#include "sweeps.hpp"
#include "team.hpp"

namespace pdyn {
namespace {

constexpr int kMaxLinks = 1 << 16;
constexpr int kMaxScanLanes = 128;  // lanes per state of the articulated-inertia and forward-dynamics scans
constexpr int kMaxFdSegments = 16;  // team forward dynamics: 16 chains x 16 lanes + 2 wavefronts per workgroup
constexpr int kBlock = 64;      // adjoint kernels, and the default workgroup
constexpr int kMaxBlock = 256;  // largest workgroup of the tunable kernels
constexpr size_t kStatusBytes = 256;  // status word at the start of every workspace (padded for alignment)
static_assert(kStatusNonFinite == PDYN_STATUS_NONFINITE && kStatusPivot == PDYN_STATUS_PIVOT &&
                  kStatusWait == PDYN_STATUS_WAIT,
              "status bits of the kernels and of the C ABI");
// Default kernel variant: the role split (2) for the adjoints; for forward
// dynamics and ID+FD the role split while a one-wavefront launch would leave
// SIMDs idle (up to 128 states per CU), else the one-wavefront kernel (1),
// whose fewer instructions win once every SIMD holds several wavefronts.
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Link records in T and in double (the double table serves the transforms of
// the wrench recursion).
template <class T>
__global__ void __launch_bounds__(256) k_link_table(int64_t n_links, const T* __restrict__ placement,
                                                    const T* __restrict__ twist, const T* __restrict__ inertia,
                                                    T* __restrict__ table, double* __restrict__ wtable) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_links) return;
  double rec[kLinkWords];
  make_link_record(placement + 7 * i, twist + 6 * i, inertia + 10 * i, rec);
#pragma unroll
  for (int k = 0; k < kLinkWords; ++k) {
    table[i * kLinkWords + k] = (T)rec[k];
    wtable[i * kLinkWords + k] = rec[k];
  }
}

template <class T> struct BoundaryArgs {
  T V0[6], dV0[6];
};

// One chain per state: the chain that lane index j runs (state s, its first
// link, its link count), written by the table derivation from link_ptr and
// order and clamped there, so that every kernel stays inside its tables and the
// caller's arrays whatever the device copies of link_ptr and order hold.
struct LaneChain {
  int32_t s, link0, n, pad;
};

// The chain of lane index j, clamped: an order entry outside 0 .. n_chains-1
// becomes chain 0 with no links; a chain starts inside 0 .. n_links_total and
// has at most n_max links, none past n_links_total.
__device__ __forceinline__ LaneChain clamp_chain(int64_t j, int n_chains, int n_max, int64_t n_links_total,
                                                 const int32_t* __restrict__ link_ptr,
                                                 const int32_t* __restrict__ order) {
  LaneChain lc{0, 0, 0, 0};
  const int c = order ? order[j] : (int)j;
  if (c < 0 || c >= n_chains) return lc;
  int64_t l0 = link_ptr[c], l1 = link_ptr[c + 1];
  l0 = l0 < 0 ? 0 : (l0 > n_links_total ? n_links_total : l0);
  l1 = l1 > n_links_total ? n_links_total : l1;
  int64_t len = l1 - l0;
  len = len < 0 ? 0 : (len > n_max ? n_max : len);
  lc.s = c;
  lc.link0 = (int32_t)l0;
  lc.n = (int32_t)len;
  return lc;
}

// One chain per state: the same records interleaved over the 64 lanes of each
// wavefront (the layout of IlvRec), n_max records per group of 64 lane
// indices; lane index j runs chain order[j] (chain j without an order), and
// lanes_out[j] records that chain for the kernels. Records past a chain's end
// and lanes past the last chain hold zeros. One thread per (group, record, lane).
template <class T>
__global__ void __launch_bounds__(256) k_link_table_ilv(int n_chains, int n_max, int64_t n_links_total,
                                                        const int32_t* __restrict__ link_ptr,
                                                        const int32_t* __restrict__ order,
                                                        const T* __restrict__ placement, const T* __restrict__ twist,
                                                        const T* __restrict__ inertia, T* __restrict__ table,
                                                        double* __restrict__ wtable, LaneChain* __restrict__ lanes_out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = (int)(t % 64);
  const int64_t slot = t / 64;  // group * n_max + record
  const int i = (int)(slot % n_max);
  const int64_t j = (slot / n_max) * 64 + lane;
  if (j >= ((int64_t)n_chains + 63) / 64 * 64) return;
  double rec[kLinkWords];
  bool live = false;
  if (j < n_chains) {
    const LaneChain lc = clamp_chain(j, n_chains, n_max, n_links_total, link_ptr, order);
    if (i == 0) lanes_out[j] = lc;
    if (i < lc.n) {
      const int64_t l = (int64_t)lc.link0 + i;
      make_link_record(placement + 7 * l, twist + 6 * l, inertia + 10 * l, rec);
      live = true;
    }
  }
  if (!live) {
#pragma unroll
    for (int k = 0; k < kLinkWords; ++k) rec[k] = 0.0;
  }
  constexpr int V = IlvRec<T>::V, W = IlvRec<double>::V;
  T* tp = table + slot * kLinkWords * 64 + lane * V;
  double* wp = wtable + slot * kLinkWords * 64 + lane * W;
#pragma unroll
  for (int k = 0; k < kLinkWords; ++k) {
    tp[(k / V) * 64 * V + k % V] = (T)rec[k];
    wp[(k / W) * 64 * W + k % W] = rec[k];
  }
}

struct ChainOf {
  int s, n;
  int64_t link0, dof0;
};
// The state a lane index runs and its chain. SHARED (one chain for every
// state) is a compile-time flag so that n stays wave-uniform and the link
// records load through the scalar unit; otherwise the clamped lane map.
template <bool SHARED>
__device__ __forceinline__ ChainOf chain_of(int lane_index, int n_max, const LaneChain* __restrict__ lanes) {
  ChainOf c;
  if (SHARED) {
    c.s = lane_index;
    c.n = n_max;
    c.link0 = 0;
    c.dof0 = (int64_t)lane_index * n_max;
  } else {
    const LaneChain lc = lanes[lane_index];
    c.s = lc.s;
    c.n = lc.n;
    c.link0 = lc.link0;
    c.dof0 = lc.link0;
  }
  return c;
}

// The link records a lane reads: the shared chain's, back to back (a
// wave-uniform address), or the lane's piece of its wavefront's interleaved
// block (k_link_table_ilv).
template <bool SHARED, class T>
__device__ __forceinline__ auto rec_view(const T* table, int lane_index, int n_max) {
  if constexpr (SHARED)
    return table;
  else
    return IlvRec<T>{table + ((int64_t)(lane_index / 64) * n_max * kLinkWords * 64 +
                              (int64_t)(lane_index % 64) * IlvRec<T>::V)};
}

// SHARED: one chain shared by every state, known at compile time, so that the
// link records are read with wave-uniform (scalar) loads.
template <class T, int MODE, bool SHARED, int SWEEPS = kAllSweeps>
__global__ void __launch_bounds__(kMaxBlock) k_dynamics(int n_states, int n_max,
                                                        const LaneChain* __restrict__ lanes,
                                                        const T* __restrict__ table,
                                                        const double* __restrict__ wtable, const T* q, const T* qd,
                                                        const T* qdd_in, const T* tau_in, T* tau_out, T* qdd_out,
                                                        const T* __restrict__ tip, BoundaryArgs<T> ba, T* scratch,
                                                        unsigned* status) {
  const long n_work = ((long)n_states + blockDim.x - 1) / blockDim.x;
  for (long wb = blockIdx.x; wb < n_work; wb += gridDim.x) {  // persistent when gridDim.x < n_work
    const int lane_index = (int)(wb * blockDim.x) + (int)threadIdx.x;
    if (lane_index >= n_states) continue;
    const ChainOf ch = chain_of<SHARED>(lane_index, n_max, lanes);
    const int s = ch.s, n = ch.n;
    const int64_t dof0 = ch.dof0;
    JointIO<T> io;
    io.q = q + dof0;
    io.qd = qd + dof0;
    io.qdd_in = qdd_in ? qdd_in + dof0 : nullptr;
    io.tau_in = tau_in ? tau_in + dof0 : nullptr;
    io.tau_out = tau_out ? tau_out + dof0 : nullptr;
    io.qdd_out = qdd_out ? qdd_out + dof0 : nullptr;
    Boundary<T> bd;
    bd.V0 = {v3(ba.V0[0], ba.V0[1], ba.V0[2]), v3(ba.V0[3], ba.V0[4], ba.V0[5])};
    bd.dV0 = {v3(ba.dV0[0], ba.dV0[1], ba.dV0[2]), v3(ba.dV0[3], ba.dV0[4], ba.dV0[5])};
    if (tip) {
      const T* t = tip + 6 * (int64_t)s;
      bd.Ftip = {v3(t[0], t[1], t[2]), v3(t[3], t[4], t[5])};
    } else {
      bd.Ftip = sp_zero<T>();
    }
    // scratch column = lane: consecutive lanes touch consecutive words
    Scratch<T> scr{scratch + lane_index, (long)n_states, ScratchWords<MODE>::value, status};
    // one chain per state: link records differ between lanes, so they are prefetched like the other inputs
    dynamics_one_state<T, MODE, StoreQdd<T>, FormPose<T>, SWEEPS, !SHARED>(n, rec_view<SHARED>(table, lane_index, n_max),
                                                                  rec_view<SHARED>(wtable, lane_index, n_max), io, bd, scr,
                                                                  StoreQdd<T>{io.qdd_out});
  }
}

template <class T>
__device__ __forceinline__ Boundary<T> boundary_of(const BoundaryArgs<T>& ba) {
  Boundary<T> bd;
  bd.V0 = {v3(ba.V0[0], ba.V0[1], ba.V0[2]), v3(ba.V0[3], ba.V0[4], ba.V0[5])};
  bd.dV0 = {v3(ba.dV0[0], ba.dV0[1], ba.dV0[2]), v3(ba.dV0[3], ba.dV0[4], ba.dV0[5])};
  bd.Ftip = sp_zero<T>();
  return bd;
}

// Role-split forward dynamics (variant 2): per group of 64 states, wavefront 0
// runs the articulated-body inertia pass (A), wavefront 1 the bias
// Newton-Euler pass (B1), and for ID+FD another wavefront the inverse
// dynamics, which shares nothing with A and B and ends on its own. Wavefront 1
// then runs the bias wrench / z-hat pass (B2) and the lambda pass. With
// OVERLAP two transform wavefronts (P_f, P_b, below) feed A, B1 and the
// inverse dynamics.
//
// OVERLAP: A keeps U_i, 1/D_i in LDS and publishes its progress (links done,
// counted from the tip) in an LDS word after each link; B2 follows A link by
// link instead of waiting for all of it. Only B2 waits here, and only for A,
// which never waits, so the wait always ends; its spin bound only guards
// against a broken invariant. Without OVERLAP (the chain's articulated terms do
// not fit in LDS) A writes them to global scratch and a workgroup barrier
// orders A before B2.
constexpr int kSpinLimit = 1 << 20;  // ~30 ms of s_sleep 1; a correct wait lasts one link of pass A

struct LdsProgress {
  int* p;
  __device__ void operator()(int k) const { __hip_atomic_store(p, k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP); }
};
// The same for a hand-off whose data this wavefront wrote to LDS only: the
// progress word is stored after this wavefront's LDS operations have completed
// (s_waitcnt lgkmcnt(0); a wavefront's LDS operations complete in order, so the
// entries are in LDS before the word changes), without the release store's wait
// for outstanding vector-memory loads, which would expose the latency of the
// next link's prefetched inputs at every link.
struct LdsPublish {
  int* p;
  __device__ void operator()(int k) const {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);  // no compiler reordering of the LDS writes past this point
    __builtin_amdgcn_s_waitcnt(0xC07F);       // gfx9 encoding: lgkmcnt(0), vmcnt and expcnt not waited for
    __hip_atomic_store(p, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
};
// Waits until *p >= k. Progress words only grow, so the last value read is
// kept: a wait it already covers returns without touching LDS (the acquire
// that read it orders everything released up to it).
// A wait that reaches its spin bound ORs PDYN_STATUS_WAIT into the call's
// status word (see bounded_wait), so a broken hand-off never passes silently.
struct LdsWait {
  int* p;
  unsigned* status = nullptr;
  mutable int seen = 0;
  __device__ void operator()(int k) const {
    if (k <= seen) return;
    const int v = bounded_wait([&] { return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_WORKGROUP); },
                               [] { __builtin_amdgcn_s_sleep(1); }, k, kSpinLimit, status);
    if (v >= k) seen = v;
  }
};

// With OVERLAP two more wavefronts form every joint transform: P_f base to tip
// for the passes that start at the base (B1 and the inverse dynamics, which
// then form none), and P_b tip to base for pass A, which then runs only the
// articulated-body recursion. Each order goes through its own LDS ring of
// kPoseSlots entries. Producers wait only for free slots, consumers only for
// entries, so every wait ends.
constexpr int kPoseSlots = 8;
constexpr int kPoseWordsF = 14;  // R (9), p (3), sin, cos
constexpr int kPoseWordsB = 12;  // R (9), p (3)

template <class T> __device__ __forceinline__ void put_pose(T* w, const Pose<T>& g) {
#pragma unroll
  for (int j = 0; j < 9; ++j) w[j * 64] = g.R.m[j];
  w[9 * 64] = g.p.x;
  w[10 * 64] = g.p.y;
  w[11 * 64] = g.p.z;
}
template <class T> __device__ __forceinline__ Pose<T> get_pose(const T* r) {
  Pose<T> g;
#pragma unroll
  for (int j = 0; j < 9; ++j) g.R.m[j] = r[j * 64];
  g.p = v3(r[9 * 64], r[10 * 64], r[11 * 64]);
  return g;
}

template <class T> struct RingPutF {  // base-to-tip entries
  T* ring;       // [kPoseSlots][kPoseWordsF][64 lanes]
  int* ready;    // entries written
  int* used_b;   // entries taken by B1
  int* used_id;  // entries taken by the inverse dynamics (null without it)
  int lane;
  unsigned* status;
  LdsWait wait_b{used_b, status}, wait_id{used_id, status};
  __device__ void operator()(int i, const Pose<T>& g, T sn, T cs) const {
    wait_b(i - kPoseSlots + 1);
    if (used_id) wait_id(i - kPoseSlots + 1);
    T* w = ring + (long)(i % kPoseSlots) * kPoseWordsF * 64 + lane;
    put_pose(w, g);
    w[12 * 64] = sn;
    w[13 * 64] = cs;
    LdsProgress{ready}(i + 1);
  }
};
// A pose source (see FormPose) that takes link i's entry from the base-to-tip ring.
template <class T> struct RingTakeF {
  const T* ring;
  int* ready;
  int* used;
  int lane;
  unsigned* status;
  LdsWait wait{ready, status};
  __device__ void operator()(int i, const Link<T>&, T, Pose<T>* g, T* sn, T* cs) const {
    wait(i + 1);
    const T* r = ring + (long)(i % kPoseSlots) * kPoseWordsF * 64 + lane;
    *g = get_pose(r);
    *sn = r[12 * 64];
    *cs = r[13 * 64];
    LdsProgress{used}(i + 1);
  }
};
// Pass C's entries, base to tip, written by two producers (even links, odd
// links) that each bump their own ready word: link i waits for ready[i % 2].
template <class T> struct RingTakeF2 {
  const T* ring;
  int* ready;  // [2]
  int* used;
  int lane;
  unsigned* status;
  LdsWait wait0{ready, status}, wait1{ready + 1, status};
  __device__ void operator()(int i, const Link<T>&, T, Pose<T>* g, T* sn, T* cs) const {
    if (i & 1)
      wait1(i + 1);
    else
      wait0(i + 1);
    const T* r = ring + (long)(i % kPoseSlots) * kPoseWordsF * 64 + lane;
    *g = get_pose(r);
    *sn = r[12 * 64];
    *cs = r[13 * 64];
    LdsProgress{used}(i + 1);
  }
};
// The adjoint sweep's hand-off: (Abar_i, Vbar_i, ybar_i) of the k-th link from
// the tip, from the recursion wavefront to the one that forms the outputs.
constexpr int kBackWords = 18;
template <class T> struct RingPutBack {
  T* ring;  // [kPoseSlots][kBackWords][64 lanes]
  int* ready;
  int* used;
  int lane;
  unsigned* status;
  LdsWait wait{used, status};
  __device__ void operator()(int k, const Sp<T>& a, const Sp<T>& v, const Sp<T>& y) const {
    wait(k - kPoseSlots + 1);
    T* w = ring + (long)(k % kPoseSlots) * kBackWords * 64 + lane;
    const Sp<T> e[3] = {a, v, y};
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      w[(6 * j + 0) * 64] = e[j].a.x;
      w[(6 * j + 1) * 64] = e[j].a.y;
      w[(6 * j + 2) * 64] = e[j].a.z;
      w[(6 * j + 3) * 64] = e[j].b.x;
      w[(6 * j + 4) * 64] = e[j].b.y;
      w[(6 * j + 5) * 64] = e[j].b.z;
    }
    LdsProgress{ready}(k + 1);
  }
};
template <class T> struct RingGetBack {
  const T* ring;
  int* ready;
  int* used;
  int lane;
  unsigned* status;
  LdsWait wait{ready, status};
  __device__ void operator()(int k, Sp<T>* a, Sp<T>* v, Sp<T>* y) const {
    wait(k + 1);
    const T* r = ring + (long)(k % kPoseSlots) * kBackWords * 64 + lane;
    Sp<T>* e[3] = {a, v, y};
#pragma unroll
    for (int j = 0; j < 3; ++j)
      *e[j] = {v3(r[(6 * j + 0) * 64], r[(6 * j + 1) * 64], r[(6 * j + 2) * 64]),
               v3(r[(6 * j + 3) * 64], r[(6 * j + 4) * 64], r[(6 * j + 5) * 64])};
    LdsProgress{used}(k + 1);
  }
};

// Pass C's epilogue in LDS: qdd_i into word 0 of link i's articulated entry.
template <class T> struct StashQdd {
  Scratch<T> abi;
  __device__ void operator()(int i, T qdd) const { abi.at(i, 0) = qdd; }
};
template <class T> struct RingPutB {  // tip-to-base entries for pass A
  T* ring;  // [kPoseSlots][kPoseWordsB][64 lanes]
  int* ready;
  int* used;
  int lane;
  unsigned* status;
  LdsWait wait{used, status};
  __device__ void operator()(int k, const Pose<T>& g) const {
    wait(k - kPoseSlots + 1);
    put_pose(ring + (long)(k % kPoseSlots) * kPoseWordsB * 64 + lane, g);
    LdsProgress{ready}(k + 1);
  }
};
template <class T> struct RingGetB {
  const T* ring;
  int* ready;
  int lane;
  unsigned* status;
  LdsWait wait{ready, status};
  __device__ Pose<T> operator()(int k) const {
    wait(k + 1);
    return get_pose(ring + (long)(k % kPoseSlots) * kPoseWordsB * 64 + lane);
  }
};

template <class T, int MODE, bool SHARED, int LDSMODE>
__global__ void __launch_bounds__(320) k_dynamics_split(int n_states, int n_max, const LaneChain* __restrict__ lanes,
                                                        const T* __restrict__ table,
                                                        const double* __restrict__ wtable, const T* q, const T* qd,
                                                        const T* qdd_in, const T* tau_in, T* tau_out, T* qdd_out,
                                                        const T* __restrict__ tip, BoundaryArgs<T> ba, T* scr_id,
                                                        T* scr_bias, T* scr_abi, unsigned* status) {
  // LDSMODE: 0 no LDS hand-off (barrier); 1 U_i, 1/D_i in LDS and the
  // transform wavefronts with their rings; 2 U_i alone in LDS (B2 forms 1/D_i,
  // so that longer chains fit); 3 as 1, and B1's bias wrenches handed to B2 in
  // LDS too instead of through HBM. LDS: [link][kAbiLds][64 lanes], then (modes
  // 1, 3) the two rings, then (mode 3) the bias wrenches [link][6][64].
  constexpr bool OVERLAP = LDSMODE != 0;
  constexpr bool kRings = LDSMODE == 1 || LDSMODE == 3;
  constexpr bool kFhatLds = LDSMODE == 3;
  constexpr int kAbiLds = kRings ? kAbiWords : 6;
  extern __shared__ __align__(16) unsigned char lds_abi[];
  __shared__ int progress, ready_f, used_b, used_id, ready_b, used_a, ready_l[2], used_l;
  if (OVERLAP) {
    if (threadIdx.x == 0) {
      progress = 0;
      ready_f = 0;
      used_b = 0;
      used_id = 0;
      ready_b = 0;
      used_a = 0;
      ready_l[0] = 0;
      ready_l[1] = 0;
      used_l = 0;
    }
    __syncthreads();
  }
  // roles: 0 articulated inertia (A), 1 bias passes (B), then with the rings
  // 2 transforms base to tip (P_f), 3 transforms tip to base (P_b) and
  // 4 inverse dynamics, else 2 inverse dynamics
  constexpr bool kWithID = MODE == kModeIDFD;
  constexpr int kRoleID = kRings ? 4 : 2;
  const int role = threadIdx.x / 64;  // wave-uniform
  const int lane = (int)(threadIdx.x % 64);
  const int lane_index = blockIdx.x * 64 + lane;
  const bool active = lane_index < n_states;
  // with a shared chain n stays uniform, so link records load through the scalar unit
  int s = 0, n = SHARED ? n_max : 0;
  int64_t dof0 = 0;
  if (active) {
    const ChainOf ch = chain_of<SHARED>(lane_index, n_max, lanes);
    s = ch.s;
    n = ch.n;
    dof0 = ch.dof0;
  }
  // links of the wavefront's longest chain: the last value of its progress words
  int n_wave = n;
  if (!SHARED) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) n_wave = max(n_wave, __shfl_xor(n_wave, o));
  }
  const auto tab = rec_view<SHARED>(table, lane_index, n_max);
  const auto wtab = rec_view<SHARED>(wtable, lane_index, n_max);
  Boundary<T> bd = boundary_of(ba);
  if (active && tip) {
    const T* t = tip + 6 * (int64_t)s;
    bd.Ftip = {v3(t[0], t[1], t[2]), v3(t[3], t[4], t[5])};
  }
  const Scratch<T> abi = OVERLAP ? Scratch<T>{reinterpret_cast<T*>(lds_abi) + lane, 64L, kAbiLds, status}
                                 : Scratch<T>{scr_abi + lane_index, (long)n_states, kAbiWords, status};
  const Scratch<T> bias{scr_bias + lane_index, (long)n_states, kBiasWords, status};
  const SPtr<const T> qs(q + dof0), qds(qd + dof0);
  T* const ring_f = reinterpret_cast<T*>(lds_abi) + (long)n_max * kAbiLds * 64;
  T* const ring_b = ring_f + (long)kPoseSlots * kPoseWordsF * 64;
  const Scratch<T> fhat_lds{ring_b + (long)kPoseSlots * kPoseWordsB * 64 + lane, 64L, 6, status};
  const Scratch<T>* const fhat = kFhatLds ? &fhat_lds : nullptr;
  // Pass C takes the transforms again through the base-to-tip ring, once B1
  // and the inverse dynamics have taken every entry: P_f forms the even links,
  // P_b (idle by then) the odd ones.
  if (kRings && role == 2) {
    if (active) {
      split_pose_fwd(n, tab, qs, RingPutF<T>{ring_f, &ready_f, &used_b, kWithID ? &used_id : nullptr, lane, status});
      LdsWait{&used_b, status}(n_wave);
      if (kWithID) LdsWait{&used_id, status}(n_wave);
      split_pose_fwd(n, tab, qs, RingPutF<T>{ring_f, &ready_l[0], &used_l, nullptr, lane, status}, 0, 2);
    }
    return;
  }
  if (kRings && role == 3) {
    if (active) {
      split_pose_bwd(n, tab, wtab, qs, RingPutB<T>{ring_b, &ready_b, &used_a, lane, status});
      LdsWait{&used_b, status}(n_wave);
      if (kWithID) LdsWait{&used_id, status}(n_wave);
      split_pose_fwd(n, tab, qs, RingPutF<T>{ring_f, &ready_l[1], &used_l, nullptr, lane, status}, 1, 2);
    }
    return;
  }
  if (role == kRoleID) {
    // inverse dynamics: ends here; a workgroup barrier waits only for wavefronts still running
    if (active) {
      JointIO<T> io{qs, qds, SPtr<const T>(qdd_in + dof0), SPtr<const T>(), SPtr<T>(tau_out + dof0), SPtr<T>()};
      const Scratch<T> idscr{scr_id + lane_index, (long)n_states, ScratchWords<kModeID>::value, status};
      if (kRings)
        dynamics_one_state<T, kModeID>(n, tab, wtab, io, bd, idscr, StoreQdd<T>{SPtr<T>()},
                                       RingTakeF<T>{ring_f, &ready_f, &used_id, lane, status});
      else
        dynamics_one_state<T, kModeID, StoreQdd<T>, FormPose<T>, kAllSweeps, !SHARED>(n, tab, wtab, io, bd, idscr,
                                                                                    StoreQdd<T>{SPtr<T>()});
    }
    return;
  }
  if (active) {
    if (role == 0) {
      if (kRings)
        split_abi_from_poses(n, tab, abi, RingGetB<T>{ring_b, &ready_b, lane, status}, LdsProgress{&used_a},
                             LdsProgress{&progress});
      else if (OVERLAP)
        split_abi_pass<T, LdsProgress, !SHARED>(n, tab, wtab, qs, abi, LdsProgress{&progress});
      else
        split_abi_pass<T, NoHandoff, !SHARED>(n, tab, wtab, qs, abi);
    } else {
      if (kRings)
        split_bias_forward(n, tab, qs, qds, bd, bias, RingTakeF<T>{ring_f, &ready_f, &used_b, lane, status}, fhat);
      else
        split_bias_forward<T, FormPose<T>, !SHARED>(n, tab, qs, qds, bd, bias);
    }
  }
  if (!OVERLAP) __syncthreads();
  if (active && role == 1) {
    if (kRings)
      split_bias_backward<T, LdsWait, !SHARED, true>(n, tab, wtab, qs, SPtr<const T>(tau_in + dof0), bd, bias,
                                                     abi, LdsWait{&progress, status}, fhat);
    else if (OVERLAP)
      split_bias_backward<T, LdsWait, !SHARED>(n, tab, wtab, qs, SPtr<const T>(tau_in + dof0), bd, bias, abi,
                                               LdsWait{&progress, status});
    else
      split_bias_backward<T, NoHandoff, !SHARED>(n, tab, wtab, qs, SPtr<const T>(tau_in + dof0), bd, bias, abi);
    if (kRings) {
      // pass C runs out of LDS alone: qdd_i goes to word 0 of link i's entry (read by then), then out
      split_lambda<T, StashQdd<T>, !SHARED, true>(n, tab, qs, bias, abi, StashQdd<T>{abi},
                                                 RingTakeF2<T>{ring_f, ready_l, &used_l, lane, status});
      T* const out = qdd_out + dof0;
      for (int i = 0; i < n; ++i) out[i] = abi.at(i, 0);
    } else
      split_lambda<T, StoreQdd<T>, !SHARED>(n, tab, qs, bias, abi, StoreQdd<T>{SPtr<T>(qdd_out + dof0)});
  }
}

// Role-split inverse dynamics (variant 2): per group of 64 states, wavefront 1
// (P_f) forms the joint transforms base to tip and hands them through an LDS
// ring to wavefront 0, which runs the two Newton-Euler sweeps without forming
// any. P_f waits only for free slots and wavefront 0 only for entries.
template <class T, bool SHARED>
__global__ void __launch_bounds__(128) k_id_split(int n_states, int n_max, const LaneChain* __restrict__ lanes,
                                                  const T* __restrict__ table,
                                                  const double* __restrict__ wtable, const T* q, const T* qd,
                                                  const T* qdd_in, T* tau_out, const T* __restrict__ tip,
                                                  BoundaryArgs<T> ba, T* scratch, unsigned* status) {
  __shared__ T ring[kPoseSlots * kPoseWordsF * 64];
  __shared__ int ready, used;
  if (threadIdx.x == 0) {
    ready = 0;
    used = 0;
  }
  __syncthreads();
  const int role = threadIdx.x / 64;  // wave-uniform
  const int lane = (int)(threadIdx.x % 64);
  const int lane_index = blockIdx.x * 64 + lane;
  const bool active = lane_index < n_states;
  int s = 0, n = SHARED ? n_max : 0;
  int64_t dof0 = 0;
  if (active) {
    const ChainOf ch = chain_of<SHARED>(lane_index, n_max, lanes);
    s = ch.s;
    n = ch.n;
    dof0 = ch.dof0;
  }
  const auto tab = rec_view<SHARED>(table, lane_index, n_max);
  const auto wtab = rec_view<SHARED>(wtable, lane_index, n_max);
  const SPtr<const T> qs(q + dof0);
  if (role == 1) {
    if (active) split_pose_fwd(n, tab, qs, RingPutF<T>{ring, &ready, &used, nullptr, lane, status});
    return;
  }
  if (!active) return;
  Boundary<T> bd = boundary_of(ba);
  if (tip) {
    const T* t = tip + 6 * (int64_t)s;
    bd.Ftip = {v3(t[0], t[1], t[2]), v3(t[3], t[4], t[5])};
  }
  JointIO<T> io{qs, SPtr<const T>(qd + dof0), SPtr<const T>(qdd_in + dof0), SPtr<const T>(), SPtr<T>(tau_out + dof0),
                SPtr<T>()};
  const Scratch<T> scr{scratch + lane_index, (long)n_states, ScratchWords<kModeID>::value, status};
  dynamics_one_state<T, kModeID>(n, tab, wtab, io, bd, scr, StoreQdd<T>{SPtr<T>()},
                                 RingTakeF<T>{ring, &ready, &used, lane, status});
}

// ---- team kernels: P lanes per chain, segmented scans (team.hpp) ---------------------
//
// Lane index L runs member k = L % P of team j = L / P; team j takes state j
// (in lane order) and member k the k-th segment of its chain. The cross-lane
// scans below move an operand between the lanes of a team word by word with
// wave shuffles (ds_bpermute), log2(P) steps (Kogge-Stone).

template <int P, class Op> __device__ __forceinline__ Op team_shfl_up(const Op& x, int d) {
  static_assert(sizeof(Op) % 4 == 0, "operands are made of 32-bit words");
  constexpr int W = sizeof(Op) / 4;
  unsigned w[W];
  __builtin_memcpy(w, &x, sizeof(Op));
#pragma unroll
  for (int i = 0; i < W; ++i) w[i] = (unsigned)__shfl_up((int)w[i], (unsigned)d, P);
  Op r;
  __builtin_memcpy(&r, w, sizeof(Op));
  return r;
}
template <int P, class Op> __device__ __forceinline__ Op team_shfl_down(const Op& x, int d) {
  constexpr int W = sizeof(Op) / 4;
  unsigned w[W];
  __builtin_memcpy(w, &x, sizeof(Op));
#pragma unroll
  for (int i = 0; i < W; ++i) w[i] = (unsigned)__shfl_down((int)w[i], (unsigned)d, P);
  Op r;
  __builtin_memcpy(&r, w, sizeof(Op));
  return r;
}
// Exclusive prefix over the team, later (+) earlier: member k gets the
// composite of members 0 .. k-1 (member 0: `id`). Every lane of the wave must
// take part.
template <int P, class Op, class Comb>
__device__ __forceinline__ Op team_prefix_exclusive(Op x, int k, const Op& id, const Comb& comb) {
#pragma unroll
  for (int d = 1; d < P; d <<= 1) {
    const Op y = team_shfl_up<P>(x, d);
    if (k >= d) x = comb(x, y);
  }
  const Op e = team_shfl_up<P>(x, 1);
  return k == 0 ? id : e;
}
// Exclusive suffix over the team, earlier (x) later: member k gets the
// composite of members k+1 .. P-1 (the last member: `id`).
template <int P, class Op, class Comb>
__device__ __forceinline__ Op team_suffix_exclusive(Op x, int k, const Op& id, const Comb& comb) {
#pragma unroll
  for (int d = 1; d < P; d <<= 1) {
    const Op y = team_shfl_down<P>(x, d);
    if (k + d < P) x = comb(x, y);
  }
  const Op e = team_shfl_down<P>(x, 1);
  return k == P - 1 ? id : e;
}

// Inverse dynamics by the two segmented scans (variant 4). Scratch: per lane,
// the slots of its segment, [slot][kTeamIdWords][n_lanes].
template <class T, int P, bool SHARED>
__global__ void __launch_bounds__(256) k_id_team(int n_states, int n_max, const LaneChain* __restrict__ lanes,
                                                 const T* __restrict__ table, const double* __restrict__ wtable,
                                                 const T* q, const T* qd, const T* qdd_in, T* tau_out,
                                                 const T* __restrict__ tip, BoundaryArgs<T> ba, T* scratch,
                                                 long n_lanes, unsigned* status) {
  const long L = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = (int)(L / P), k = (int)(L % P);
  const bool active = j < n_states;
  ChainOf ch{0, 0, 0, 0};
  if (active) ch = chain_of<SHARED>(j, n_max, lanes);
  const Seg sg = segment_of(ch.n, P, k);
  const auto tab = rec_view<SHARED>(table, j, n_max);
  const auto wtab = rec_view<SHARED>(wtable, j, n_max);
  const SPtr<const T> qs(q + ch.dof0), qds(qd + ch.dof0), qdds(qdd_in + ch.dof0);
  Boundary<T> bd = boundary_of(ba);
  if (active && tip) {
    const T* t = tip + 6 * (int64_t)ch.s;
    bd.Ftip = {v3(t[0], t[1], t[2]), v3(t[3], t[4], t[5])};
  }
  const Scratch<T> scr{scratch + L, n_lanes, kTeamIdWords, status};
  const FwdOp<T> agg = team_fwd_aggregate(sg, tab, qs, qds, qdds, bd);
  const FwdOp<T> pre = team_prefix_exclusive<P>(agg, k, fwd_identity<T>(),
                                                [](const FwdOp<T>& a, const FwdOp<T>& b) { return fwd_combine(a, b); });
  Sp<T> dV = bd.dV0, V = bd.V0;
  if (k > 0) {
    dV = pre.x1;
    V = pre.x2;
  }
  team_fwd_apply(sg, tab, qs, qds, qdds, dV, V, scr);
  const BwdOp<double> bag = team_bwd_aggregate(sg, wtab, qs, scr);
  const BwdOp<double> suf = team_suffix_exclusive<P>(
      bag, k, bwd_identity<double>(), [](const BwdOp<double>& a, const BwdOp<double>& b) { return bwd_combine(a, b); });
  team_bwd_apply(sg, wtab, qs, scr, bwd_apply(suf, cast_sp<double>(bd.Ftip)), SPtr<T>(tau_out + ch.dof0));
}

// ---- joint-space inertia (jsiia.hpp) -----------------------------------------------
//
// One lane per state of a shared chain, grid-stride. FD: qdd = M^-1 (tau - tau_bias);
// otherwise M(q) only, written whole to M ([n_states][n][n]). Working storage:
// [jsiia_words(n)][n_states] doubles (consecutive lanes, consecutive words).
template <class T, bool FD, bool SOLVE = true>
__global__ void __launch_bounds__(256) k_jsiia(int n_states, int n, const T* __restrict__ table,
                                               const double* __restrict__ wtable, const T* q, const T* qd,
                                               const T* tau, T* qdd, T* M, const T* __restrict__ tip,
                                               BoundaryArgs<T> ba, double* work, unsigned* status) {
  const int stride = gridDim.x * blockDim.x;
  for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < n_states; s += stride) {
    Boundary<T> bd = boundary_of(ba);
    if (tip) {
      const T* t = tip + 6 * (int64_t)s;
      bd.Ftip = {v3(t[0], t[1], t[2]), v3(t[3], t[4], t[5])};
    }
    const JsiiaWork<SPtr<double>> ws{SPtr<double>(work + s, (long)n_states), n};
    const int64_t row = (int64_t)s * n;
    T* const Ms = M ? M + row * n : nullptr;
    auto mout = [&](int i, int k, double v) {
      if (!FD) Ms[(int64_t)i * n + k] = (T)v;
    };
    jsiia_mass_matrix<T, FD>(n, table, wtable, SPtr<const T>(q + row), SPtr<const T>(FD ? qd + row : nullptr),
                             SPtr<const T>(FD ? tau + row : nullptr), bd, ws, mout);
    if (FD && SOLVE) {
      unsigned bits = 0;
      const bool ok = jsiia_solve<T>(n, ws, [&](int i, double v) {
        const T x = (T)v;
        qdd[row + i] = x;
        if (!__builtin_isfinite(x)) bits |= kStatusNonFinite;
      });
      if (!ok) bits |= kStatusPivot;
      if (bits) __hip_atomic_fetch_or(status, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// The factorisation and solves of JSIIA for n <= NT links (NT a power of two up
// to 32; longer chains keep the per-lane solve of k_jsiia): a team of NT lanes per state, lane i holding row i of M (the packed
// lower triangle that k_jsiia left in `work`) in registers. Right-looking
// Cholesky: at step j lane j's diagonal becomes L_jj, the lanes below scale
// their entry of column j, and every entry of the trailing rows takes its
// update from column j, whose entries reach the other lanes by wave shuffles.
// Then L y = tau-hat with y_k broadcast the same way, and L^T qdd = y with the
// columns of L read from LDS, where each lane leaves its row. Double throughout.
template <class T, int NT>
__global__ void __launch_bounds__(256) k_jsiia_chol(int n_states, int n, const double* __restrict__ work, T* qdd,
                                                    unsigned* status) {
  extern __shared__ __align__(16) unsigned char lds_chol[];
  const long L = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long s = L / NT;
  const int i = (int)(L % NT);
  const bool active = s < n_states;
  const bool row = active && i < n;
  double* const Ls = reinterpret_cast<double*>(lds_chol) + (long)(threadIdx.x / NT) * NT * NT;
  const long area = 13L * n;  // jsiia.hpp: poses (12 n), tau-hat (n), then the packed triangle
  const long stride = n_states;
  const double* const w = work + (active ? s : 0);
  double r[NT];
#pragma unroll
  for (int k = 0; k < NT; ++k) r[k] = (row && k <= i) ? w[(area + (long)i * (i + 1) / 2 + k) * stride] : 0.0;
  double b = row ? w[(12L * n + i) * stride] : 0.0;
  bool ok = true;
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    if (j < n) {
      const double d = __shfl(r[j], j, NT);
      if (i == j && !(d > 0.0)) ok = false;
      const double ljj = sqrt(d);
      if (i == j) r[j] = ljj;
      else if (i > j) r[j] = r[j] / ljj;
#pragma unroll
      for (int k = j + 1; k < NT; ++k) {
        if (k < n) {
          const double lkj = __shfl(r[j], k, NT);
          if (i >= k) r[k] -= r[j] * lkj;
        }
      }
    }
  }
  // L y = tau-hat: lane k finishes y_k, then every lane below takes its term
#pragma unroll
  for (int k = 0; k < NT; ++k) {
    if (k < n) {
      if (i == k) b = b / r[k];
      const double yk = __shfl(b, k, NT);
      if (i > k) b -= r[k] * yk;
    }
  }
  // L^T qdd = y: column k of L is row k's entries, read from LDS
#pragma unroll
  for (int k = 0; k < NT; ++k) Ls[(long)i * NT + k] = r[k];
  __syncthreads();
  for (int k = n - 1; k >= 0; --k) {
    if (i == k) b = b / Ls[(long)k * NT + k];
    const double xk = __shfl(b, k, NT);
    if (i < k) b -= Ls[(long)k * NT + i] * xk;
  }
  if (row) {
    const T x = (T)b;
    qdd[s * n + i] = x;
    unsigned bits = 0;
    if (!__builtin_isfinite(x)) bits |= kStatusNonFinite;
    if (!ok) bits |= kStatusPivot;
    if (bits) __hip_atomic_fetch_or(status, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Forward dynamics (and ID+FD) by the team scans (variant 4). A workgroup takes
// C chains (in lane order; C chosen on the host so that their per-link values
// fit in LDS, at most kTeamChains) and has three kinds of wavefronts:
//  * team wavefronts, P lanes per chain (team.hpp): first every link transform
//    of their segments into LDS (then one add to `pdone`); then the velocities
//    and bias accelerations by the segmented forward scan, leaving the bias
//    wrench Fhat_i of every link in their global slots (then one add to
//    `p1done`); for ID+FD then the inverse dynamics;
//  * A, one lane per chain: the articulated-body recursion (7), serial, from
//    the transforms in LDS, publishing its progress in `aprog` after each link;
//  * Z, one lane per chain: once the team's Fhat are in, the bias wrench and
//    z-hat / c-hat tip to base as one recursion (folded eq. (20)), each link as
//    soon as A has it, then lambda / qdd base to tip; qdd is written out at the end.
// No workgroup barrier follows the first: waits are one-directional (A waits
// for the team, Z for the team and A), so every wavefront runs to its end.
constexpr int kTeamChains = 16;

template <class T, int MODE, int P, bool SHARED>
__global__ void __launch_bounds__(384) k_fd_team(int n_states, int n_max, int C, const LaneChain* __restrict__ lanes,
                                                 const T* __restrict__ table, const double* __restrict__ wtable,
                                                 const T* q, const T* qd, const T* qdd_in, const T* tau_in,
                                                 T* tau_out, T* qdd_out, const T* __restrict__ tip,
                                                 BoundaryArgs<T> ba, T* scr_id, T* scr_bias, long n_lanes,
                                                 unsigned* status) {
  extern __shared__ __align__(16) unsigned char lds_team[];
  __shared__ int pdone, p1done, aprog;
  if (threadIdx.x == 0) {
    pdone = 0;
    p1done = 0;
    aprog = 0;
  }
  __syncthreads();
  const int team_lanes = C * P;
  const int team_waves = (team_lanes + 63) / 64;
  const int wave = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
  Boundary<T> bd = boundary_of(ba);
  if (wave < team_waves) {
    const int t = (int)threadIdx.x;
    const int k = t % P, c = t / P;
    const long j = (long)blockIdx.x * C + c;
    const bool active = t < team_lanes && j < n_states;
    const int jj = active ? (int)j : 0;
    ChainOf ch{0, 0, 0, 0};
    if (active) ch = chain_of<SHARED>(jj, n_max, lanes);
    const Seg sg = segment_of(ch.n, P, k);
    const auto tab = rec_view<SHARED>(table, jj, n_max);
    const auto wtab = rec_view<SHARED>(wtable, jj, n_max);
    const SPtr<const T> qs(q + ch.dof0), qds(qd + ch.dof0);
    const TeamChainLds<T> cl = TeamChainLds<T>::at(lds_team, n_max, C, active ? c : 0);
    team_pose_pass(sg, tab, wtab, qs, cl);
    if (lane == 0) __hip_atomic_fetch_add(&pdone, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (active && tip) {
      const T* tp = tip + 6 * (int64_t)ch.s;
      bd.Ftip = {v3(tp[0], tp[1], tp[2]), v3(tp[3], tp[4], tp[5])};
    }
    const long L = j * P + k;
    const auto fcomb = [](const FwdOp<T>& a, const FwdOp<T>& b) { return fwd_combine(a, b); };
    const auto bcomb = [](const BwdOp<double>& a, const BwdOp<double>& b) { return bwd_combine(a, b); };
    // the bias forces (qdd = 0): the forward scan leaves Fhat_bias in the team slots for Z
    {
      const Scratch<T> scr{scr_bias + L, n_lanes, kTeamIdWords, status};
      const FwdOp<T> pre =
          team_prefix_exclusive<P>(team_fwd_aggregate(sg, tab, qs, qds, SPtr<const T>(), bd), k, fwd_identity<T>(), fcomb);
      team_fwd_apply(sg, tab, qs, qds, SPtr<const T>(), k > 0 ? pre.x1 : bd.dV0, k > 0 ? pre.x2 : bd.V0, scr);
    }
    if (lane == 0) __hip_atomic_fetch_add(&p1done, 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (MODE & kModeID) {
      const Scratch<T> scr{scr_id + L, n_lanes, kTeamIdWords, status};
      const SPtr<const T> qdds(qdd_in + ch.dof0);
      const FwdOp<T> pre =
          team_prefix_exclusive<P>(team_fwd_aggregate(sg, tab, qs, qds, qdds, bd), k, fwd_identity<T>(), fcomb);
      team_fwd_apply(sg, tab, qs, qds, qdds, k > 0 ? pre.x1 : bd.dV0, k > 0 ? pre.x2 : bd.V0, scr);
      const BwdOp<double> suf =
          team_suffix_exclusive<P>(team_bwd_aggregate(sg, wtab, qs, scr), k, bwd_identity<double>(), bcomb);
      team_bwd_apply(sg, wtab, qs, scr, bwd_apply(suf, cast_sp<double>(bd.Ftip)), SPtr<T>(tau_out + ch.dof0));
    }
    return;
  }
  const int role = wave - team_waves;  // 0: articulated-body pass; 1: z-hat, then lambda
  const long j = (long)blockIdx.x * C + lane;
  const bool active = lane < C && j < n_states;
  const int jj = active ? (int)j : 0;
  ChainOf ch{0, 0, 0, 0};
  if (active) ch = chain_of<SHARED>(jj, n_max, lanes);
  const auto tab = rec_view<SHARED>(table, jj, n_max);
  const auto wtab = rec_view<SHARED>(wtable, jj, n_max);
  const TeamChainLds<T> cl = TeamChainLds<T>::at(lds_team, n_max, C, active ? lane : 0);
  if (role == 0) {
    LdsWait{&pdone, status}(team_waves);
    if (active) {
      const int n = ch.n;
      const auto get = [&](int k) { return cl.pose(n - 1 - k); };  // the k-th transform from the tip
      split_abi_from_poses<T, decltype(get), NoHandoff, LdsPublish, decltype(tab), !SHARED>(
          n, tab, cl.abi(status), get, NoHandoff(), LdsPublish{&aprog});
    }
    return;
  }
  LdsWait{&p1done, status}(team_waves);
  if (!active) return;
  Sp<double> Ftip = sp_zero<double>();
  if (tip) {
    const T* tp = tip + 6 * (int64_t)ch.s;
    Ftip = {v3((double)tp[0], (double)tp[1], (double)tp[2]), v3((double)tp[3], (double)tp[4], (double)tp[5])};
  }
  // the team's slot of link i: member i / len, slot i % len, [slot][8][n_lanes] from the chain's first lane
  const int len = (ch.n + P - 1) / P;
  const long team0 = j * P;
  const auto fhat = [&](int i) {
    const int k = i / len;
    const T* f = scr_bias + (long)(i - k * len) * kTeamIdWords * n_lanes + team0 + k;
    return Sp<T>{v3(f[0], f[n_lanes], f[2 * n_lanes]), v3(f[3 * n_lanes], f[4 * n_lanes], f[5 * n_lanes])};
  };
  team_bias_zhat_pass(ch.n, wtab, SPtr<const T>(q + ch.dof0), SPtr<const T>(tau_in + ch.dof0), cl, fhat, Ftip,
                      LdsWait{&aprog, status});
  team_lambda_pass(ch.n, tab, cl, Scratch<T>{nullptr, 0L, 0, status});
  T* const out = qdd_out + ch.dof0;
  for (int i = 0; i < ch.n; ++i) out[i] = cl.chat(i);
}

// ---- adjoints ------------------------------------------------------------------
//
// One lane per state as above. With a shared chain each lane writes its
// inertia-parameter cotangents to its own column of [link][10][state]
// (consecutive lanes, consecutive words) and k_reduce_lanes sums the columns
// in a fixed order, so the result is deterministic. With one chain per state
// each lane writes its own links directly.

enum : int { kVjpID = 0, kVjpFD = 1 };
enum : int { kPiNone = 0, kPiLanes = 1, kPiDirect = 2 };

template <class T, int PI> struct PiSink {
  T* out;        // kPiLanes: this lane's column of [link][10][n_lanes]; kPiDirect: [links of this chain][10]
  long stride;   // kPiLanes: n_lanes
  __device__ void put(int i, const T g[10]) {
    if (PI == kPiLanes) {
#pragma unroll
      for (int k = 0; k < 10; ++k) out[((long)i * 10 + k) * stride] = g[k];
    } else if (PI == kPiDirect) {
#pragma unroll
      for (int k = 0; k < 10; ++k) out[(long)i * 10 + k] = g[k];
    }
  }
};

// Scratch of the adjoints: [n_max][kVjpWords][n_states].
template <class T, int OP, int PI, bool SHARED>
__global__ void __launch_bounds__(kBlock) k_vjp(int n_states, int n_max, const LaneChain* __restrict__ lanes,
                                                const T* __restrict__ table,
                                                const double* __restrict__ wtable, const T* q, const T* qd,
                                                const T* qdd, const T* bar_in, T* q_bar, T* qd_bar, T* qdd_bar,
                                                T* tau_bar, T* pi_out, const T* __restrict__ tip, BoundaryArgs<T> ba,
                                                T* scratch, unsigned* status) {
  const int lane_index = blockIdx.x * blockDim.x + threadIdx.x;
  if (lane_index >= n_states) return;
  const ChainOf c = chain_of<SHARED>(lane_index, n_max, lanes);
  const int s = c.s;
  VjpIO<T> io;
  io.q = q + c.dof0;
  io.qd = qd + c.dof0;
  io.qdd = qdd + c.dof0;
  io.bar_in = bar_in + c.dof0;
  io.q_bar = q_bar + c.dof0;
  io.qd_bar = qd_bar + c.dof0;
  io.qdd_bar = (OP == kVjpID) ? qdd_bar + c.dof0 : nullptr;
  io.tau_bar = (OP == kVjpFD) ? tau_bar + c.dof0 : nullptr;
  Boundary<T> bd = boundary_of(ba);
  if (tip) {
    const T* t = tip + 6 * (int64_t)s;
    bd.Ftip = {v3(t[0], t[1], t[2]), v3(t[3], t[4], t[5])};
  }
  Scratch<T> scr{scratch + lane_index, (long)n_states, kVjpWords, status};
  PiSink<T, PI> sink;
  sink.out = nullptr;
  sink.stride = 0;
  if (PI == kPiLanes) {
    sink.out = pi_out + lane_index;
    sink.stride = n_states;
  } else if (PI == kPiDirect) {
    sink.out = pi_out + c.link0 * 10;
  }
  const auto tab = rec_view<SHARED>(table, lane_index, n_max);
  const auto wtab = rec_view<SHARED>(wtable, lane_index, n_max);
  if (OP == kVjpID) id_vjp_one_state(c.n, tab, wtab, io, bd, scr, sink);
  else fd_vjp_one_state(c.n, tab, wtab, io, bd, scr, sink);
}

// Role-split adjoint (variant 2): per group of 64 states, wavefront X runs the
// Fbar recursion (and for FD first the articulated-body solve for u), while
// wavefront Y runs the Newton-Euler sweeps (V, A, Fhat, then F); after one
// workgroup barrier X forms the inertia-parameter cotangents and Y runs the
// tip-to-base adjoint sweep. Scratch: Y's [n_max][kVjpWords][n_states], X's
// [n_max][kVjpXWords][n_states].
//
// OVERLAP (ID adjoint, when the wrenches fit in LDS): X's Fbar pass also hands
// its transforms to Y's Newton-Euler pass through an LDS ring; after the
// barrier X runs the wrench sweep, writing F_i to LDS with a progress word,
// and Y's adjoint sweep follows it link by link. X then forms the
// inertia-parameter cotangents.
// OVERLAP (FD adjoint, when the articulated terms fit in LDS): a third
// wavefront A runs the articulated-body pass (U_i, 1/D_i into LDS with a
// progress word) and X's solve follows it, keeping z-hat and c-hat only; a
// fourth, P_b, forms A's transforms and hands them over through a ring.
// OVERLAP == 2 (when one more ring fits): the adjoint sweep is cut in two
// after the barrier. Y runs its recursion and hands (Abar_i, Vbar_i, ybar_i)
// through an LDS ring to the third wavefront (A for FD, a wavefront of its
// own for ID), which forms q_bar, qd_bar and qdd_bar link by link. For ID, X
// runs the wrench sweep and a fourth wavefront the inertia-parameter
// cotangents; for FD, X runs the cotangents.
template <class T, int OP, int PI, bool SHARED, int OVERLAP>
__global__ void __launch_bounds__(256) k_vjp_split(int n_states, int n_max, const LaneChain* __restrict__ lanes,
                                                   const T* __restrict__ table,
                                                   const double* __restrict__ wtable, const T* q, const T* qd,
                                                   const T* qdd, const T* bar_in, T* q_bar, T* qd_bar, T* qdd_bar,
                                                   T* tau_bar, T* pi_out, const T* __restrict__ tip,
                                                   BoundaryArgs<T> ba, T* scratch, T* xscratch,
                                                   unsigned* status) {
  constexpr bool kOv = OVERLAP >= 1 && OP == kVjpID;  // ID: ring and wrench hand-offs
  constexpr bool kAw = OVERLAP >= 1 && OP == kVjpFD;  // FD: the articulated-body wavefront A
  constexpr bool kCut = OVERLAP == 2;                 // the adjoint sweep on two wavefronts
  // kOv: ring, then F [n_max][6][64]; kAw: U_i, 1/D_i [n_max][kAbiWords][64], then P_b's ring
  // [kPoseSlots][kPoseWordsB][64]; then (kCut) the (Abar, Vbar, ybar) ring [kPoseSlots][kBackWords][64]
  extern __shared__ __align__(16) unsigned char lds_vjp[];
  __shared__ int ready, used, fprog, aprog, bready, bused, pready, pused, qready, qused;
  if (kOv || kAw) {
    if (threadIdx.x == 0) {
      ready = 0;
      used = 0;
      fprog = 0;
      aprog = 0;
      bready = 0;
      bused = 0;
      pready = 0;
      pused = 0;
      qready = 0;
      qused = 0;
    }
    __syncthreads();
  }
  // wave-uniform: 0 = X, 1 = Y, 2 = A (kAw) or the outputs (kCut), 3 = P_b (kAw) or, for ID with
  // kCut, the inertia-parameter cotangents
  const int role = threadIdx.x / 64;
  const int lane = (int)(threadIdx.x % 64);
  const int lane_index = blockIdx.x * 64 + lane;
  const bool active = lane_index < n_states;
  int s = 0, n = SHARED ? n_max : 0;
  int64_t link0 = 0, dof0 = 0;
  if (active) {
    const ChainOf ch = chain_of<SHARED>(lane_index, n_max, lanes);
    s = ch.s;
    n = ch.n;
    link0 = ch.link0;
    dof0 = ch.dof0;
  }
  const auto tab = rec_view<SHARED>(table, lane_index, n_max);
  const auto wtab = rec_view<SHARED>(wtable, lane_index, n_max);
  Boundary<T> bd = boundary_of(ba);
  if (active && tip) {
    const T* t = tip + 6 * (int64_t)s;
    bd.Ftip = {v3(t[0], t[1], t[2]), v3(t[3], t[4], t[5])};
  }
  const Scratch<T> scr{scratch + lane_index, (long)n_states, kVjpWords, status};
  const Scratch<T> xs{xscratch + lane_index, (long)n_states, kVjpXWords, status};
  const SPtr<const T> qs(q + dof0), qds(qd + dof0), qdds(qdd + dof0), bar(bar_in + dof0);
  T* const ring = reinterpret_cast<T*>(lds_vjp);
  const Scratch<T> fl{ring + (long)kPoseSlots * kPoseWordsF * 64 + lane, 64L, 6, status};
  const Scratch<T> abi{reinterpret_cast<T*>(lds_vjp) + lane, 64L, kAbiWords, status};
  T* const pring = reinterpret_cast<T*>(lds_vjp) + (long)n_max * kAbiWords * 64;
  T* const bring = reinterpret_cast<T*>(lds_vjp) +
                   (kOv ? ((long)kPoseSlots * kPoseWordsF + (long)n_max * 6) * 64
                        : (long)n_max * kAbiWords * 64 + (long)kPoseSlots * kPoseWordsB * 64);
  if (kAw && role == 3) {
    if (active) split_pose_bwd(n, tab, wtab, qs, RingPutB<T>{pring, &pready, &pused, lane, status});
    // without the cut sweep it ends here; the workgroup barrier waits only for wavefronts still running
    if (!kCut) return;
  }
  if (kAw && role == 2) {
    if (active)
      split_abi_from_poses(n, tab, abi, RingGetB<T>{pring, &pready, lane, status}, LdsProgress{&pused},
                           LdsProgress{&aprog});
    // without the cut sweep it ends here
    if (!kCut) return;
  }
  if (active && role < 2) {
    if (role == 0) {
      if (kOv)
        vjp_fbar_pass(n, tab, qs, bar, T(1), xs, RingPutF<T>{ring, &ready, &used, nullptr, lane, status});
      else if (OP == kVjpID)
        vjp_fbar_pass(n, tab, qs, bar, T(1), xs);
      else if (kAw)
        fdvjp_solve_with_abi(n, tab, wtab, qs, bar, SPtr<T>(tau_bar + dof0), xs, abi, LdsWait{&aprog, status});
      else
        fdvjp_solve_pass(n, tab, wtab, qs, bar, SPtr<T>(tau_bar + dof0), xs);
    } else {
      if (kOv)
        vjp_ne_forward(n, tab, qs, qds, qdds, bd, scr, RingTakeF<T>{ring, &ready, &used, lane, status});
      else
        vjp_newton_euler_pass(n, tab, wtab, qs, qds, qdds, bd, scr);
    }
  }
  __syncthreads();
  if (!active) return;
  if (kCut) {
    const SPtr<T> qddb = OP == kVjpID ? SPtr<T>(qdd_bar + dof0) : SPtr<T>();
    // FD: P_b forms the transforms of Y's recursion again, tip to base, through its ring (A took every
    // entry of the first round before the barrier)
    if (kAw && role == 3) {
      split_pose_bwd_sc(n, tab, qs, RingPutB<T>{pring, &qready, &qused, lane, status});
      return;
    }
    // the inertia-parameter cotangents: X's for FD, a fourth wavefront's for ID (beside X's wrench sweep)
    if ((role == 0 && kAw) || role == 3) {
      if (PI != kPiNone) {
        PiSink<T, PI> sink;
        sink.out = (PI == kPiLanes) ? pi_out + lane_index : pi_out + link0 * 10;
        sink.stride = (PI == kPiLanes) ? n_states : 1;
        vjp_inertia_pass(n, tab, xs, scr, sink);
      }
    } else if (role == 0) {
      vjp_wrench_pass(n, wtab, qs, bd, scr, fl, LdsProgress{&fprog});
    } else if (role == 1) {
      if (kAw)
        vjp_back_recursion(n, tab, qs, qds, xs, scr, RingPutBack<T>{bring, &bready, &bused, lane, status},
                           RingGetB<T>{pring, &qready, lane, status}, LdsProgress{&qused});
      else
        vjp_back_recursion(n, tab, qs, qds, xs, scr, RingPutBack<T>{bring, &bready, &bused, lane, status});
    } else {
      PiSink<T, kPiNone> sink;  // the inertia cotangents are X's
      const RingGetBack<T> get{bring, &bready, &bused, lane, status};
      if (kOv)
        vjp_back_outputs(n, tab, qds, qdds, xs, scr, SPtr<T>(q_bar + dof0), SPtr<T>(qd_bar + dof0), qddb, fl,
                         LdsWait{&fprog, status}, get, sink);
      else
        vjp_back_outputs(n, tab, qds, qdds, xs, scr, SPtr<T>(q_bar + dof0), SPtr<T>(qd_bar + dof0), qddb, scr,
                         NoHandoff(), get, sink);
    }
    return;
  }
  if (role == 0) {
    if (kOv) vjp_wrench_pass(n, wtab, qs, bd, scr, fl, LdsProgress{&fprog});
    if (PI != kPiNone) {
      PiSink<T, PI> sink;
      sink.out = (PI == kPiLanes) ? pi_out + lane_index : pi_out + link0 * 10;
      sink.stride = (PI == kPiLanes) ? n_states : 1;
      vjp_inertia_pass(n, tab, xs, scr, sink);
    }
  } else {
    const SPtr<T> qddb = OP == kVjpID ? SPtr<T>(qdd_bar + dof0) : SPtr<T>();
    if (kOv)
      vjp_back_pass(n, tab, qs, qds, qdds, xs, scr, SPtr<T>(q_bar + dof0), SPtr<T>(qd_bar + dof0), qddb, fl,
                    LdsWait{&fprog, status});
    else
      vjp_back_pass(n, tab, qs, qds, qdds, xs, scr, SPtr<T>(q_bar + dof0), SPtr<T>(qd_bar + dof0), qddb, scr);
  }
}

// The plain form of the adjoints (variant 3): the passes of k_vjp_split at its
// lowest LDS level, each as its own launch of one wavefront per 64 states, with
// every per-link intermediate in the workspace (HBM) between launches:
//   PASS 0  the cotangent recursion F-bar (ID), or the articulated-body solve
//           u = M^-1 qdd_bar and F-bar (FD);
//   PASS 1  Newton-Euler sweep 1 (V, A, Fhat);   PASS 2  the wrench sweep (F);
//   PASS 3  the inertia-parameter cotangents;    PASS 4  the tip-to-base adjoint sweep.
enum : int { kVjpPassX = 0, kVjpPassNeFwd = 1, kVjpPassWrench = 2, kVjpPassInertia = 3, kVjpPassBack = 4 };

template <class T, int OP, int PI, bool SHARED, int PASS>
__global__ void __launch_bounds__(64) k_vjp_pass(int n_states, int n_max, const LaneChain* __restrict__ lanes,
                                                 const T* __restrict__ table, const double* __restrict__ wtable,
                                                 const T* q, const T* qd, const T* qdd, const T* bar_in, T* q_bar,
                                                 T* qd_bar, T* qdd_bar, T* tau_bar, T* pi_out,
                                                 const T* __restrict__ tip, BoundaryArgs<T> ba, T* scratch,
                                                 T* xscratch, unsigned* status) {
  const int lane_index = blockIdx.x * 64 + (int)threadIdx.x;
  if (lane_index >= n_states) return;
  const ChainOf ch = chain_of<SHARED>(lane_index, n_max, lanes);
  const int n = ch.n;
  const auto tab = rec_view<SHARED>(table, lane_index, n_max);
  const auto wtab = rec_view<SHARED>(wtable, lane_index, n_max);
  Boundary<T> bd = boundary_of(ba);
  if (tip) {
    const T* t = tip + 6 * (int64_t)ch.s;
    bd.Ftip = {v3(t[0], t[1], t[2]), v3(t[3], t[4], t[5])};
  }
  const Scratch<T> scr{scratch + lane_index, (long)n_states, kVjpWords, status};
  const Scratch<T> xs{xscratch + lane_index, (long)n_states, kVjpXWords, status};
  const SPtr<const T> qs(q + ch.dof0), qds(qd + ch.dof0), qdds(qdd + ch.dof0), bar(bar_in + ch.dof0);
  if (PASS == kVjpPassX) {
    if (OP == kVjpID)
      vjp_fbar_pass(n, tab, qs, bar, T(1), xs);
    else
      fdvjp_solve_pass(n, tab, wtab, qs, bar, SPtr<T>(tau_bar + ch.dof0), xs);
  } else if (PASS == kVjpPassNeFwd) {
    vjp_ne_forward(n, tab, qs, qds, qdds, bd, scr);
  } else if (PASS == kVjpPassWrench) {
    vjp_wrench_pass(n, wtab, qs, bd, scr, scr);
  } else if (PASS == kVjpPassInertia) {
    PiSink<T, PI> sink;
    sink.out = (PI == kPiLanes) ? pi_out + lane_index : pi_out + ch.link0 * 10;
    sink.stride = (PI == kPiLanes) ? n_states : 1;
    vjp_inertia_pass(n, tab, xs, scr, sink);
  } else {
    const SPtr<T> qddb = OP == kVjpID ? SPtr<T>(qdd_bar + ch.dof0) : SPtr<T>();
    vjp_back_pass(n, tab, qs, qds, qdds, xs, scr, SPtr<T>(q_bar + ch.dof0), SPtr<T>(qd_bar + ch.dof0), qddb, scr);
  }
}

// out[i] = sum over j < n_in of in[i * n_in + j], one workgroup per output, fixed
// order (strided partial sums in double, then a fixed tree), so deterministic.
template <class T>
__global__ void __launch_bounds__(256) k_reduce_lanes(int n_in, const T* __restrict__ in, T* __restrict__ out) {
  __shared__ double part[256];
  const long i = blockIdx.x;
  double acc = 0.0;
  for (int j = threadIdx.x; j < n_in; j += 256) acc += (double)in[i * n_in + j];
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[i] = (T)part[0];
}

// ---- rollouts -------------------------------------------------------------------

template <class T> struct DevRows {  // row t of a [T][dofs] array, offset to this state
  const T* base;
  long stride;
  __device__ const T* operator()(int t) const { return base + (long)t * stride; }
};
template <class T> struct DevMutRows {
  T* base;
  long stride;
  __device__ T* operator()(int t) const { return base + (long)t * stride; }
};
template <class T> struct DevCkpt {
  T* qb;
  T* qdb;
  long stride;
  __device__ T* q(int c) const { return qb + (long)c * stride; }
  __device__ T* qd(int c) const { return qdb + (long)c * stride; }
};
// pi_bar accumulated over steps: element (link i, parameter k) at acc[(10 i + k) * stride].
template <class T> struct AccumSink {
  T* acc;
  long stride;
  __device__ void put(int i, const T g[10]) {
#pragma unroll
    for (int k = 0; k < 10; ++k) acc[(10L * i + k) * stride] += g[k];
  }
};
struct NoSink {
  template <class T> __device__ void put(int, const T*) {}
};

// Forward rollout, one lane per state, all steps in one launch.
template <class T, bool SHARED>
__global__ void __launch_bounds__(kMaxBlock) k_rollout(int n_states, int n_max, const LaneChain* __restrict__ lanes,
                                                       const T* __restrict__ table,
                                                       const double* __restrict__ wtable, int steps, T dt, int every,
                                                       const T* tau_seq, T* q, T* qd, T* ckpt_q, T* ckpt_qd, long dofs,
                                                       BoundaryArgs<T> ba, T* scratch, unsigned* status) {
  const long n_work = ((long)n_states + blockDim.x - 1) / blockDim.x;
  for (long wb = blockIdx.x; wb < n_work; wb += gridDim.x) {
    const int lane_index = (int)(wb * blockDim.x) + (int)threadIdx.x;
    if (lane_index >= n_states) continue;
    const ChainOf c = chain_of<SHARED>(lane_index, n_max, lanes);
    Scratch<T> scr{scratch + lane_index, (long)n_states, ScratchWords<kModeFD>::value, status};
    rollout_one_state(c.n, rec_view<SHARED>(table, lane_index, n_max), rec_view<SHARED>(wtable, lane_index, n_max), steps, dt, every,
                      SPtr<T>(q + c.dof0), SPtr<T>(qd + c.dof0), DevRows<T>{tau_seq + c.dof0, dofs},
                      DevCkpt<T>{ckpt_q + c.dof0, ckpt_qd + c.dof0, dofs}, boundary_of(ba), scr);
  }
}

// Adjoint of a rollout, one lane per state. Workspace regions, all
// lane-interleaved: adjoint scratch [n_max][kVjpWords][n_states]; working rows
// [(3 every + 6) n_max][n_states]; pi accumulators [n_max][10][n_states]
// (shared chain; zeroed here).
template <class T, int PI, bool SHARED>
__global__ void __launch_bounds__(kBlock) k_rollout_vjp(int n_states, int n_max, const LaneChain* __restrict__ lanes,
                                                        const T* __restrict__ table,
                                                        const double* __restrict__ wtable, int steps, T dt, int every,
                                                        const T* tau_seq, const T* ckpt_q, const T* ckpt_qd,
                                                        const T* qT_bar, const T* qdT_bar, T* q0_bar, T* qd0_bar,
                                                        T* tau_bar_seq, T* pi_out, long dofs, BoundaryArgs<T> ba,
                                                        T* scratch, T* rows_ws, T* pi_acc, unsigned* status) {
  const int lane_index = blockIdx.x * blockDim.x + threadIdx.x;
  if (lane_index >= n_states) return;
  const ChainOf c = chain_of<SHARED>(lane_index, n_max, lanes);
  // working rows, lane-interleaved: element i of row r at rows_ws[(r n_max + i) n_states + lane]
  const long S = n_states;
  T* const rb = rows_ws + lane_index;
  auto row = [&](int r) { return SPtr<T>(rb + (long)r * n_max * S, S); };
  RolloutRows<T> rows{SPtr<T>(rb, S), SPtr<T>(q0_bar + c.dof0), SPtr<T>(qd0_bar + c.dof0), row(3 * every),
                      row(3 * every + 1), row(3 * every + 2), row(3 * every + 3), row(3 * every + 4),
                      row(3 * every + 5), n_max};
  for (int i = 0; i < c.n; ++i) {
    rows.lq[i] = qT_bar[c.dof0 + i];
    rows.lqd[i] = qdT_bar[c.dof0 + i];
  }
  Scratch<T> scr{scratch + lane_index, (long)n_states, kVjpWords, status};
  DevRows<T> tau{tau_seq + c.dof0, dofs};
  DevCkpt<T> ck{const_cast<T*>(ckpt_q) + c.dof0, const_cast<T*>(ckpt_qd) + c.dof0, dofs};
  DevMutRows<T> tb{tau_bar_seq + c.dof0, dofs};
  const auto tab = rec_view<SHARED>(table, lane_index, n_max);
  const auto wtab = rec_view<SHARED>(wtable, lane_index, n_max);
  if (PI == kPiNone) {
    NoSink sink;
    rollout_vjp_one_state(c.n, tab, wtab, steps, dt, every, tau, ck, tb, rows, boundary_of(ba), scr, sink);
  } else {
    AccumSink<T> sink;
    if (PI == kPiLanes) {  // shared chain: a private column per state, summed afterwards
      sink.acc = pi_acc + lane_index;
      sink.stride = n_states;
    } else {  // one chain per state: its own rows of the output
      sink.acc = pi_out + c.link0 * 10;
      sink.stride = 1;
    }
    for (int i = 0; i < 10 * c.n; ++i) sink.acc[(long)i * sink.stride] = T(0);
    rollout_vjp_one_state(c.n, tab, wtab, steps, dt, every, tau, ck, tb, rows, boundary_of(ba), scr, sink);
  }
}

// One semi-implicit Euler step in place, n joint values (one thread each,
// grid-stride): qd <- qd + dt qdd, then q <- q + dt qd with the new qd.
template <class T>
__global__ void __launch_bounds__(256) k_euler_step(int64_t n, T dt, T* __restrict__ q, T* __restrict__ qd,
                                                    const T* __restrict__ qdd) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const T v = qd[i] + dt * qdd[i];
    qd[i] = v;
    q[i] = q[i] + dt * v;
  }
}

// Adjoint of k_euler_step for a reverse pass that alternates with the
// forward-dynamics adjoint: first the forward-dynamics cotangents of the later
// step are added (qb += qbf, qdb += qdbf, pib += pibf, each if given), then the
// step's own adjoint: qdb <- qdb + dt qb (the cotangent of qd before the step),
// qddb = dt qdb (the cotangent of qdd). qb passes through unchanged.
template <class T>
__global__ void __launch_bounds__(256) k_euler_step_vjp(int64_t n, T dt, T* __restrict__ qb, T* __restrict__ qdb,
                                                        const T* __restrict__ qbf, const T* __restrict__ qdbf,
                                                        T* __restrict__ qddb, int64_t n_pi, T* __restrict__ pib,
                                                        const T* __restrict__ pibf) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    T a = qb[i], b = qdb[i];
    if (qbf) {
      a += qbf[i];
      b += qdbf[i];
      qb[i] = a;
    }
    if (qddb) {
      b += dt * a;
      qddb[i] = dt * b;
    }
    qdb[i] = b;
  }
  if (pibf)
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pi; i += stride) pib[i] += pibf[i];
}

// ---- Jacobian mode -----------------------------------------------------------------
//
// Row j of the Jacobian of y = f(x) is the vector-Jacobian product with the
// one-hot cotangent e_j. For a chunk of states of a shared chain, row
// r = s n + j of the expanded batch is a copy of state s with cotangent e_j, so
// the adjoint kernels, run over the expanded batch, write J[s][j][k] directly
// ([states][n][n] row-major, like [rows][n]).
template <class T>
__global__ void __launch_bounds__(256) k_jac_expand(int64_t rows, int n, const T* q, const T* qd, const T* x3,
                                                    const T* tip, T* eq, T* eqd, T* ex3, T* ebar, T* etip) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < rows * n; e += stride) {
    const int64_t r = e / n;
    const int k = (int)(e % n);
    const int64_t src = (r / n) * n + k;
    eq[e] = q[src];
    eqd[e] = qd[src];
    ex3[e] = x3[src];
    ebar[e] = (k == (int)(r % n)) ? T(1) : T(0);
  }
  if (tip)
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < rows * 6; e += stride)
      etip[e] = tip[(e / 6) / n * 6 + e % 6];
}

// ---- host side ------------------------------------------------------------------

struct Layout {
  size_t table_off, wtable_off, scratch_off, scratch_bytes, partial_off, xscratch_off, total;
};

int scratch_words(int op) {
  switch (op) {
    case PDYN_OP_RNEA_ID: return ScratchWords<kModeID>::value;
    case PDYN_OP_ABA_FD: return ScratchWords<kModeFD>::value;
    case PDYN_OP_ID_FD: return ScratchWords<kModeIDFD>::value;
    case PDYN_OP_RNEA_ID_VJP:
    case PDYN_OP_ABA_FD_VJP: return kVjpWords;
    case PDYN_OP_JSIIA_FD:
    case PDYN_OP_MASS_MATRIX: return 0;  // their own layout, jsiia_words doubles per state
    default: return -1;
  }
}

bool is_vjp(int op) { return op == PDYN_OP_RNEA_ID_VJP || op == PDYN_OP_ABA_FD_VJP; }
bool is_jsiia(int op) { return op == PDYN_OP_JSIIA_FD || op == PDYN_OP_MASS_MATRIX; }

// The host copies of the CSR offsets and of the lane order (pdyn_model): first
// offset 0, every chain 1 .. n_links_max links, last offset n_links_total, and
// the order a permutation. Runs before any device work.
int check_host_csr(const pdyn_model* m) {
  if (m->n_chains == 1) return PDYN_OK;
  const int32_t* lp = m->link_ptr_host;
  if (!lp || lp[0] != 0) return PDYN_EINVAL;
  for (int32_t c = 0; c < m->n_chains; ++c) {
    const int64_t len = (int64_t)lp[c + 1] - lp[c];
    if (len < 1 || len > m->n_links_max) return PDYN_EINVAL;
  }
  if ((int64_t)lp[m->n_chains] != m->n_links_total) return PDYN_EINVAL;
  if (m->order) {
    if (!m->order_host) return PDYN_EINVAL;
    std::vector<unsigned char> seen((size_t)m->n_chains, 0);
    for (int32_t j = 0; j < m->n_chains; ++j) {
      const int32_t c = m->order_host[j];
      if (c < 0 || c >= m->n_chains || seen[(size_t)c]) return PDYN_EINVAL;
      seen[(size_t)c] = 1;
    }
  }
  return PDYN_OK;
}

int check_model_batch(const pdyn_model* m, const pdyn_batch* b) {
  if (!m || !b) return PDYN_EINVAL;
  if (m->n_chains < 1 || m->n_links_max < 1 || m->n_links_total < 1 || b->n_states < 0) return PDYN_EINVAL;
  if (!m->placement || !m->twist || !m->inertia) return PDYN_EINVAL;
  if (m->n_links_max > kMaxLinks) return PDYN_EUNSUPPORTED;
  if (b->block_threads < 0 || b->block_threads % 64 != 0 || b->block_threads > kMaxBlock) return PDYN_EINVAL;
  if (b->max_blocks < 0) return PDYN_EINVAL;
  if (b->variant < 0 || b->variant > 4) return PDYN_EINVAL;
  if (b->segments < 0 || b->segments > 64 || (b->segments & (b->segments - 1))) return PDYN_EINVAL;
  if (m->order && (m->n_chains == 1 || (uintptr_t)m->order % sizeof(int32_t) != 0)) return PDYN_EINVAL;
  if (m->n_chains == 1) {
    if (m->n_links_total != m->n_links_max) return PDYN_EINVAL;
  } else {
    if (m->n_chains != b->n_states || !m->link_ptr) return PDYN_EINVAL;
    if (m->n_links_total > INT32_MAX) return PDYN_EUNSUPPORTED;
    // a call without prepared tables derives them from link_ptr and order: check their host copies
    if (!m->prepared) return check_host_csr(m);
  }
  return PDYN_OK;
}

// The derived tables: records in the scalar type, then the same in double.
// One shared chain: [n][32] each. One chain per state: interleaved over the
// lanes of each wavefront, n_max records per group of 64 lane indices
// ([group][n_max][32][64] each, see k_link_table_ilv), then the clamped lane
// map [n_chains] (LaneChain) that the kernels use with these tables.
size_t ilv_slots(const pdyn_model* m) { return ((size_t)m->n_chains + 63) / 64 * (size_t)m->n_links_max; }
size_t tables_bytes(const pdyn_model* m, size_t scalar, size_t* wtable_off, size_t* lanes_off = nullptr) {
  const size_t recs = m->n_chains == 1 ? (size_t)m->n_links_total : ilv_slots(m) * 64;
  const size_t t = align_up(recs * kLinkWords * scalar);
  const size_t w = align_up(recs * kLinkWords * sizeof(double));
  if (wtable_off) *wtable_off = t;
  if (lanes_off) *lanes_off = t + w;
  return t + w + (m->n_chains == 1 ? 0 : align_up((size_t)m->n_chains * sizeof(LaneChain)));
}

// Lane -> chain map of the kernels: none with a shared chain; with one chain
// per state, the copy that the table derivation wrote beside the tables it
// built (so that the tables and the map always agree).
const LaneChain* lane_map(const pdyn_model* m, const char* tbase, size_t scalar) {
  if (m->n_chains == 1) return nullptr;
  size_t woff, loff;
  tables_bytes(m, scalar, &woff, &loff);
  return reinterpret_cast<const LaneChain*>(tbase + loff);
}

// Lanes per chain of the team kernels (variant 4): the batch's `segments`, or
// by default the largest power of two up to 64 that leaves at least 8 links
// per segment (at least 1 lane).
int team_lanes(const pdyn_model* m, const pdyn_batch* b, int op = PDYN_OP_RNEA_ID) {
  if (b->segments > 0) return b->segments;
  const int cap = (op == PDYN_OP_ABA_FD || op == PDYN_OP_ID_FD) ? kMaxFdSegments : 64;
  int P = 1;
  while (P < cap && m->n_links_max >= 16 * P) P *= 2;
  return P;
}

// Global scratch of the team forward-dynamics kernel: the team slots of the
// inverse dynamics (ID+FD only), then of the bias forces, [len][8][n_states * P]
// each. The per-chain values of the serial passes live in LDS.
struct FdTeamLayout {
  size_t id_off, bias_off, total;
};
FdTeamLayout fd_team_layout(int op, size_t nm, size_t B, size_t P, size_t scalar) {
  FdTeamLayout t;
  const size_t team = align_up((nm + P - 1) / P * (size_t)kTeamIdWords * B * P * scalar);
  t.id_off = 0;
  t.bias_off = op == PDYN_OP_ID_FD ? team : 0;
  t.total = t.bias_off + team;
  return t;
}

int layout_for(int op, const pdyn_model* m, const pdyn_batch* b, size_t scalar, Layout* L) {
  int words = scratch_words(op);
  if (words < 0) return PDYN_EINVAL;
  size_t woff;
  size_t tb = tables_bytes(m, scalar, &woff);
  L->table_off = 0;
  L->wtable_off = woff;
  L->scratch_off = m->prepared ? 0 : tb;
  const size_t nm = (size_t)m->n_links_max;
  L->scratch_bytes = align_up(nm * (size_t)words * (size_t)b->n_states * scalar);
  if (b->variant == 4) {  // the team kernels: their own per-segment slots, one column per lane
    const size_t P = (size_t)team_lanes(m, b, op);
    size_t need = align_up((nm + P - 1) / P * (size_t)kTeamIdWords * (size_t)b->n_states * P * scalar);
    if (op == PDYN_OP_ABA_FD || op == PDYN_OP_ID_FD) need = fd_team_layout(op, nm, b->n_states, P, scalar).total;
    if (need > L->scratch_bytes) L->scratch_bytes = need;
  }
  if (is_jsiia(op)) L->scratch_bytes = align_up((size_t)jsiia_words((int)nm) * (size_t)b->n_states * sizeof(double));
  if (op == PDYN_OP_ABA_FD || op == PDYN_OP_ID_FD) {  // room for the role-split variant too
    const size_t need = align_up(nm * (size_t)ScratchWords<kModeID>::value * (size_t)b->n_states * scalar) +
                        align_up(nm * (size_t)kBiasWords * (size_t)b->n_states * scalar) +
                        align_up(nm * (size_t)kAbiWords * (size_t)b->n_states * scalar);
    if (need > L->scratch_bytes) L->scratch_bytes = need;
  }
  if (is_vjp(op)) {
    // then the per-lane inertia cotangents [n_max][10][n_states] (shared chain),
    // then the second scratch of the role-split adjoint [n_max][kVjpXWords][n_states]
    L->partial_off = L->scratch_off + L->scratch_bytes;
    L->xscratch_off = L->partial_off + align_up(nm * 10 * (size_t)b->n_states * scalar);
    L->total = L->xscratch_off + align_up(nm * (size_t)kVjpXWords * (size_t)b->n_states * scalar);
  } else {
    L->partial_off = 0;
    L->xscratch_off = 0;
    L->total = L->scratch_off + L->scratch_bytes;
  }
  L->total += kStatusBytes;
  return PDYN_OK;
}

bool aligned(const void* p, size_t a) { return ((uintptr_t)p % a) == 0; }

// ---- launch tuning table (pdyn_load_tuning) ----------------------------------------
//
// Entries written by the autotuner: for an operation, scalar size, model kind
// (shared chain or one chain per state), a link count and a batch size, the
// launch fields of pdyn_batch to use when a call leaves all of them at 0. A
// call takes the entry of its operation, scalar size and kind whose link count
// and batch size are nearest in log scale, if both lie within a factor of 2.
struct TuneEntry {
  int op, scalar, shared, n_max, n_states, block, max_blocks, variant, segments;
};

std::mutex g_tune_mutex;
std::shared_ptr<const std::vector<TuneEntry>> g_tune;

// A minimal reader for the one document shape pdyn_load_tuning accepts:
// {"entries": [{"key": integer, ...}, ...]} (whitespace anywhere; nothing else).
struct JsonReader {
  const char* p;
  void ws() {
    while (*p == ' ' || *p == '\n' || *p == '\t' || *p == '\r') ++p;
  }
  bool lit(char c) {
    ws();
    if (*p != c) return false;
    ++p;
    return true;
  }
  bool str(std::string* out) {
    ws();
    if (*p != '"') return false;
    const char* q = ++p;
    while (*p && *p != '"' && *p != '\\') ++p;
    if (*p != '"') return false;
    out->assign(q, p);
    ++p;
    return true;
  }
  bool integer(long* out) {
    ws();
    char* end = nullptr;
    const long v = std::strtol(p, &end, 10);
    if (end == p) return false;
    p = end;
    *out = v;
    return true;
  }
};

bool valid_launch(int block, int max_blocks, int variant, int segments) {
  return block >= 0 && block % 64 == 0 && block <= kMaxBlock && max_blocks >= 0 && variant >= 0 && variant <= 4 &&
         segments >= 0 && segments <= 64 && (segments & (segments - 1)) == 0;
}

int parse_tuning(const char* text, std::vector<TuneEntry>* out) {
  JsonReader r{text};
  std::string key;
  if (!r.lit('{') || !r.str(&key) || key != "entries" || !r.lit(':') || !r.lit('[')) return PDYN_EINVAL;
  if (!r.lit(']')) {
    do {
      if (!r.lit('{')) return PDYN_EINVAL;
      TuneEntry e{-1, 0, -1, 0, -1, 0, 0, 0, 0};
      do {
        long v;
        if (!r.str(&key) || !r.lit(':') || !r.integer(&v) || v < INT32_MIN || v > INT32_MAX) return PDYN_EINVAL;
        const int iv = (int)v;
        if (key == "op") e.op = iv;
        else if (key == "scalar") e.scalar = iv;
        else if (key == "shared") e.shared = iv;
        else if (key == "n_max") e.n_max = iv;
        else if (key == "n_states") e.n_states = iv;
        else if (key == "block") e.block = iv;
        else if (key == "max_blocks") e.max_blocks = iv;
        else if (key == "variant") e.variant = iv;
        else if (key == "segments") e.segments = iv;
        else return PDYN_EINVAL;
      } while (r.lit(','));
      if (!r.lit('}')) return PDYN_EINVAL;
      if (e.op < PDYN_OP_RNEA_ID || e.op > PDYN_OP_MASS_MATRIX || (e.scalar != 4 && e.scalar != 8) ||
          (e.shared != 0 && e.shared != 1) || e.n_max < 1 || e.n_states < 0 ||
          !valid_launch(e.block, e.max_blocks, e.variant, e.segments))
        return PDYN_EINVAL;
      out->push_back(e);
    } while (r.lit(','));
    if (!r.lit(']')) return PDYN_EINVAL;
  }
  if (!r.lit('}')) return PDYN_EINVAL;
  r.ws();
  return *r.p == '\0' ? PDYN_OK : PDYN_EINVAL;
}

// The batch a call runs with: the caller's, or, when it leaves every launch
// field at 0, the tuning table's nearest entry for this call (if any).
pdyn_batch tuned_batch(int op, const pdyn_model* m, const pdyn_batch* b, size_t scalar) {
  pdyn_batch r = *b;
  if (b->block_threads || b->max_blocks || b->variant || b->segments) return r;
  std::shared_ptr<const std::vector<TuneEntry>> tab;
  {
    std::lock_guard<std::mutex> lock(g_tune_mutex);
    tab = g_tune;
  }
  if (!tab) return r;
  const int shared = m->n_chains == 1 ? 1 : 0;
  const TuneEntry* best = nullptr;
  double best_d = 0;
  for (const TuneEntry& e : *tab) {
    if (e.op != op || e.scalar != (int)scalar || e.shared != shared) continue;
    const double dn = std::fabs(std::log2((double)m->n_links_max / e.n_max));
    const double db = std::fabs(std::log2(((double)b->n_states + 1) / ((double)e.n_states + 1)));
    if (dn > 1.0 || db > 1.0) continue;
    if (!best || dn + db < best_d) {
      best = &e;
      best_d = dn + db;
    }
  }
  if (best) {
    r.block_threads = best->block;
    r.max_blocks = best->max_blocks;
    r.variant = best->variant;
    r.segments = best->segments;
  }
  return r;
}

// Workgroup size and count of the tunable kernels (validated in check_model_batch).
void launch_shape(const pdyn_batch* b, unsigned* grid, unsigned* block) {
  const unsigned bt = b->block_threads > 0 ? (unsigned)b->block_threads : (unsigned)kBlock;
  unsigned g = (unsigned)((b->n_states + bt - 1) / bt);
  if (b->max_blocks > 0 && g > (unsigned)b->max_blocks) g = (unsigned)b->max_blocks;
  *grid = g > 0 ? g : 1;
  *block = bt;
}

template <class T>
int check_ptrs(std::initializer_list<const void*> ptrs) {
  for (const void* p : ptrs)
    if (!p) return PDYN_EINVAL;
  for (const void* p : ptrs)
    if (!aligned(p, sizeof(T))) return PDYN_EALIGN;
  return PDYN_OK;
}

template <class T>
int launch_link_table(const pdyn_model* m, char* dst, hipStream_t s) {
  size_t woff, ooff;
  tables_bytes(m, sizeof(T), &woff, &ooff);
  if (m->n_chains == 1) {
    int64_t nl = m->n_links_total;
    unsigned grid = (unsigned)((nl + 255) / 256);
    hipLaunchKernelGGL(k_link_table<T>, dim3(grid), dim3(256), 0, s, nl, static_cast<const T*>(m->placement),
                       static_cast<const T*>(m->twist), static_cast<const T*>(m->inertia),
                       reinterpret_cast<T*>(dst), reinterpret_cast<double*>(dst + woff));
  } else {
    if (!m->link_ptr) return PDYN_EINVAL;
    const size_t threads = ilv_slots(m) * 64;
    if ((threads + 255) / 256 > 0x7fffffffu) return PDYN_EUNSUPPORTED;
    hipLaunchKernelGGL(k_link_table_ilv<T>, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, m->n_chains,
                       m->n_links_max, (int64_t)m->n_links_total, m->link_ptr, m->order,
                       static_cast<const T*>(m->placement), static_cast<const T*>(m->twist),
                       static_cast<const T*>(m->inertia), reinterpret_cast<T*>(dst),
                       reinterpret_cast<double*>(dst + woff), reinterpret_cast<LaneChain*>(dst + ooff));
  }
  if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
  return PDYN_OK;
}

// Compute units of the current device (queried once per device).
int cu_count() {
  static int cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cached[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) return 0;
    cached[dev] = v;
  }
  return cached[dev];
}

int pick_variant(const pdyn_batch* b, bool forward) {
  if (b->variant) return (!forward && b->variant == 4) ? 1 : b->variant;
  if (!forward) return 2;
  return (int64_t)b->n_states <= (int64_t)128 * cu_count() ? 2 : 1;
}

// Largest LDS allocation of one workgroup on the current device (queried once per device).
size_t max_lds_bytes() {
  static int cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
  if (cached[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) return 0;
    cached[dev] = v;
  }
  return (size_t)cached[dev] - 1024;  // room for the kernel's static LDS
}

// One word of device memory: zero it (out == nullptr) or copy it to *out.
__global__ void __launch_bounds__(64) k_status_word(unsigned* word, uint32_t* out) {
  if (threadIdx.x != 0) return;
  if (out) *out = *word;
  else *word = 0u;
}

// Chains per workgroup of the team forward-dynamics kernel: the most (up to
// kTeamChains, a power of two) whose per-link values fit in LDS; 0 if not even one.
int fd_team_chains(int n_max, size_t scalar) {
  const size_t cap = max_lds_bytes();
  for (int C = kTeamChains; C >= 1; C /= 2) {
    const size_t bytes = scalar == 4 ? TeamChainLds<float>::bytes(n_max, C) : TeamChainLds<double>::bytes(n_max, C);
    if (bytes <= cap) return C;
  }
  return 0;
}

template <class T, int MODE>
int launch_dynamics(const pdyn_model* m, const pdyn_batch* b, const Layout& L, const T* q, const T* qd,
                    const T* qdd_in, const T* tau_in, T* tau_out, T* qdd_out, char* ws, hipStream_t s);

// clear_status: zero the workspace's status word before the first kernel;
// status_out (device, or nullptr): receives the status word after the last.
template <class T, int MODE>
int run_dynamics(int op, const pdyn_model* m, const pdyn_batch* b, const T* q, const T* qd, const T* qdd_in,
                 const T* tau_in, T* tau_out, T* qdd_out, void* ws, size_t ws_bytes, void* stream,
                 bool clear_status = false, uint32_t* status_out = nullptr) {
  int st = check_model_batch(m, b);
  if (st) return st;
  const pdyn_batch bt = tuned_batch(op, m, b, sizeof(T));
  b = &bt;
  if (b->n_states == 0) return PDYN_OK;  // empty batch: nothing to do
  if (MODE & kModeID) {
    if ((st = check_ptrs<T>({q, qd, qdd_in, tau_out}))) return st;
  }
  if (MODE & kModeFD) {
    if ((st = check_ptrs<T>({q, qd, tau_in, qdd_out}))) return st;
  }
  if ((st = check_ptrs<T>({m->placement, m->twist, m->inertia}))) return st;
  if (m->prepared && !aligned(m->prepared, kAlign)) return PDYN_EALIGN;
  if (b->tip_wrench && !aligned(b->tip_wrench, sizeof(T))) return PDYN_EALIGN;
  if (!ws) return PDYN_EINVAL;
  if (!aligned(ws, kAlign)) return PDYN_EALIGN;
  Layout L;
  if ((st = layout_for(op, m, b, sizeof(T), &L))) return st;
  if (ws_bytes < L.total) return PDYN_EWORKSPACE;
  if ((MODE & kModeFD) && pick_variant(b, true) == 4 && b->segments > kMaxFdSegments) return PDYN_EUNSUPPORTED;

  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned* status = static_cast<unsigned*>(ws);  // the first kStatusBytes of every workspace
  if (clear_status) {
    hipLaunchKernelGGL(k_status_word, dim3(1), dim3(64), 0, s, status, nullptr);
    if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
  }
  st = launch_dynamics<T, MODE>(m, b, L, q, qd, qdd_in, tau_in, tau_out, qdd_out, static_cast<char*>(ws), s);
  if (st == PDYN_OK && status_out) {
    hipLaunchKernelGGL(k_status_word, dim3(1), dim3(64), 0, s, status, status_out);
    if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
  }
  return st;
}

// The kernels of one call of run_dynamics, after its checks.
template <class T, int MODE>
int launch_dynamics(const pdyn_model* m, const pdyn_batch* b, const Layout& L, const T* q, const T* qd,
                    const T* qdd_in, const T* tau_in, T* tau_out, T* qdd_out, char* ws, hipStream_t s) {
  int st = PDYN_OK;
  unsigned* status = reinterpret_cast<unsigned*>(ws);
  char* base = ws + kStatusBytes;
  T* scratch = reinterpret_cast<T*>(base + L.scratch_off);
  const char* tbase = m->prepared ? static_cast<const char*>(m->prepared) : base;
  const LaneChain* const lanes = lane_map(m, tbase, sizeof(T));
  const T* table = reinterpret_cast<const T*>(tbase + L.table_off);
  const double* wtable = reinterpret_cast<const double*>(tbase + L.wtable_off);
  if (!m->prepared) {
    if ((st = launch_link_table<T>(m, base, s))) return st;
  }
  BoundaryArgs<T> ba;
  for (int k = 0; k < 6; ++k) { ba.V0[k] = (T)b->base_vel[k]; ba.dV0[k] = (T)b->base_acc[k]; }
  const int variant = pick_variant(b, true);
  if (MODE == kModeID && variant == 4) {
    const int P = team_lanes(m, b);
    const long n_lanes = (long)b->n_states * P;
    const unsigned g = (unsigned)((n_lanes + 255) / 256);
    const T* tip = static_cast<const T*>(b->tip_wrench);
#define PDYN_LAUNCH_TEAM_ID(PP)                                                                                \
  do {                                                                                                         \
    if (m->n_chains == 1)                                                                                      \
      hipLaunchKernelGGL((k_id_team<T, PP, true>), dim3(g), dim3(256), 0, s, b->n_states, m->n_links_max, lanes, \
                         table, wtable, q, qd, qdd_in, tau_out, tip, ba, scratch, n_lanes, status);              \
    else                                                                                                       \
      hipLaunchKernelGGL((k_id_team<T, PP, false>), dim3(g), dim3(256), 0, s, b->n_states, m->n_links_max,      \
                         lanes, table, wtable, q, qd, qdd_in, tau_out, tip, ba, scratch, n_lanes, status);       \
  } while (0)
    switch (P) {
      case 1: PDYN_LAUNCH_TEAM_ID(1); break;
      case 2: PDYN_LAUNCH_TEAM_ID(2); break;
      case 4: PDYN_LAUNCH_TEAM_ID(4); break;
      case 8: PDYN_LAUNCH_TEAM_ID(8); break;
      case 16: PDYN_LAUNCH_TEAM_ID(16); break;
      case 32: PDYN_LAUNCH_TEAM_ID(32); break;
      default: PDYN_LAUNCH_TEAM_ID(64); break;
    }
#undef PDYN_LAUNCH_TEAM_ID
    if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
    return PDYN_OK;
  }
  if ((MODE & kModeFD) && variant == 4) {
    const int P = team_lanes(m, b, MODE == kModeIDFD ? PDYN_OP_ID_FD : PDYN_OP_ABA_FD);
    const size_t nm = (size_t)m->n_links_max, B = (size_t)b->n_states;
    const FdTeamLayout t = fd_team_layout(MODE == kModeIDFD ? PDYN_OP_ID_FD : PDYN_OP_ABA_FD, nm, B, (size_t)P, sizeof(T));
    const int C = fd_team_chains(m->n_links_max, sizeof(T));
    if (C < 1) return PDYN_EUNSUPPORTED;
    const size_t lds = TeamChainLds<T>::bytes(m->n_links_max, C);
    char* sc = reinterpret_cast<char*>(scratch);
    const long n_lanes = (long)b->n_states * P;
    const unsigned g = (unsigned)((b->n_states + C - 1) / C);
    const unsigned blk = 64u * (unsigned)((C * P + 63) / 64 + 2);
    const T* tip = static_cast<const T*>(b->tip_wrench);
#define PDYN_LAUNCH_TEAM_FD(PP)                                                                                   \
  do {                                                                                                            \
    const void* fn = m->n_chains == 1 ? reinterpret_cast<const void*>(&k_fd_team<T, MODE, PP, true>)              \
                                      : reinterpret_cast<const void*>(&k_fd_team<T, MODE, PP, false>);            \
    if (lds > 65536 && hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) \
      return PDYN_ELAUNCH;                                                                                        \
    if (m->n_chains == 1)                                                                                         \
      hipLaunchKernelGGL((k_fd_team<T, MODE, PP, true>), dim3(g), dim3(blk), lds, s, b->n_states, m->n_links_max, \
                         C, lanes, table, wtable, q, qd, qdd_in, tau_in, tau_out, qdd_out, tip, ba,               \
                         reinterpret_cast<T*>(sc + t.id_off), reinterpret_cast<T*>(sc + t.bias_off), n_lanes,    \
                         status);                                                                                 \
    else                                                                                                          \
      hipLaunchKernelGGL((k_fd_team<T, MODE, PP, false>), dim3(g), dim3(blk), lds, s, b->n_states, m->n_links_max, \
                         C, lanes, table, wtable, q, qd, qdd_in, tau_in, tau_out, qdd_out, tip, ba,               \
                         reinterpret_cast<T*>(sc + t.id_off), reinterpret_cast<T*>(sc + t.bias_off), n_lanes,    \
                         status);                                                                                 \
  } while (0)
    switch (P) {
      case 1: PDYN_LAUNCH_TEAM_FD(1); break;
      case 2: PDYN_LAUNCH_TEAM_FD(2); break;
      case 4: PDYN_LAUNCH_TEAM_FD(4); break;
      case 8: PDYN_LAUNCH_TEAM_FD(8); break;
      default: PDYN_LAUNCH_TEAM_FD(16); break;
    }
#undef PDYN_LAUNCH_TEAM_FD
    if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
    return PDYN_OK;
  }
  if (MODE == kModeID && variant == 2) {
    const unsigned g = (unsigned)((b->n_states + 63) / 64);
    if (m->n_chains == 1)
      hipLaunchKernelGGL((k_id_split<T, true>), dim3(g), dim3(128), 0, s, b->n_states, m->n_links_max, lanes,
                         table, wtable, q, qd, qdd_in, tau_out, static_cast<const T*>(b->tip_wrench), ba,
                         scratch, status);
    else
      hipLaunchKernelGGL((k_id_split<T, false>), dim3(g), dim3(128), 0, s, b->n_states, m->n_links_max, lanes,
                         table, wtable, q, qd, qdd_in, tau_out, static_cast<const T*>(b->tip_wrench), ba,
                         scratch, status);
    if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
    return PDYN_OK;
  }
  if ((MODE & kModeFD) && variant == 2) {
    const unsigned g = (unsigned)((b->n_states + 63) / 64);
    const size_t nm = (size_t)m->n_links_max, B = (size_t)b->n_states;
    T* scr_id = scratch;
    T* scr_bias = reinterpret_cast<T*>(reinterpret_cast<char*>(scr_id) +
                                       align_up(nm * ScratchWords<kModeID>::value * B * sizeof(T)));
    T* scr_abi = reinterpret_cast<T*>(reinterpret_cast<char*>(scr_bias) + align_up(nm * kBiasWords * B * sizeof(T)));
    // LDS hand-off of U_i with the transform rings and the bias wrenches if they fit, else of U_i with
    // the rings, else of U_i alone, else none
    const size_t lds_rings = (nm * kAbiWords + (size_t)kPoseSlots * (kPoseWordsF + kPoseWordsB)) * 64 * sizeof(T);
    const size_t lds_fhat = lds_rings + nm * 6 * 64 * sizeof(T);
    const size_t lds_abi = nm * 6 * 64 * sizeof(T);
    const size_t cap = max_lds_bytes();
    const int ldsmode = lds_fhat <= cap ? 3 : lds_rings <= cap ? 1 : (lds_abi <= cap ? 2 : 0);
    const size_t lds = ldsmode == 3 ? lds_fhat : ldsmode == 1 ? lds_rings : (ldsmode == 2 ? lds_abi : 0);
    const bool shared = m->n_chains == 1;
    // wavefronts: A, B, [P_f and P_b with the rings], [ID for ID+FD]
    const unsigned blk = 128 + (ldsmode == 1 || ldsmode == 3 ? 128 : 0) + ((MODE == kModeIDFD) ? 64 : 0);
#define PDYN_LAUNCH_SPLIT(SH, LM)                                                                                 \
  do {                                                                                                            \
    if (lds > 65536 &&                                                                                            \
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_dynamics_split<T, MODE, SH, LM>),                    \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)                  \
      return PDYN_ELAUNCH;                                                                                        \
    hipLaunchKernelGGL((k_dynamics_split<T, MODE, SH, LM>), dim3(g), dim3(blk), lds, s, b->n_states,              \
                       m->n_links_max, lanes, table, wtable, q, qd, qdd_in, tau_in, tau_out,      \
                       qdd_out, static_cast<const T*>(b->tip_wrench), ba, scr_id, scr_bias, scr_abi, status);     \
  } while (0)
    if (shared) {
      if (ldsmode == 3) PDYN_LAUNCH_SPLIT(true, 3);
      else if (ldsmode == 1) PDYN_LAUNCH_SPLIT(true, 1);
      else if (ldsmode == 2) PDYN_LAUNCH_SPLIT(true, 2);
      else PDYN_LAUNCH_SPLIT(true, 0);
    } else {
      if (ldsmode == 3) PDYN_LAUNCH_SPLIT(false, 3);
      else if (ldsmode == 1) PDYN_LAUNCH_SPLIT(false, 1);
      else if (ldsmode == 2) PDYN_LAUNCH_SPLIT(false, 2);
      else PDYN_LAUNCH_SPLIT(false, 0);
    }
#undef PDYN_LAUNCH_SPLIT
    if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
    return PDYN_OK;
  }
  unsigned grid, block;
  launch_shape(b, &grid, &block);
  if (variant == 3) {
    // the plain form: one launch per sweep, per-link intermediates in the (HBM) scratch between them
#define PDYN_LAUNCH_SWEEP(SH, SW)                                                                                 \
  hipLaunchKernelGGL((k_dynamics<T, MODE, SH, SW>), dim3(grid), dim3(block), 0, s, b->n_states,       \
                     m->n_links_max, lanes, table, wtable, q, qd, qdd_in, tau_in, tau_out, qdd_out, \
                     static_cast<const T*>(b->tip_wrench), ba, scratch, status)
    if (m->n_chains == 1) {
      PDYN_LAUNCH_SWEEP(true, kSweep1);
      PDYN_LAUNCH_SWEEP(true, kSweep2);
      if (MODE & kModeFD) PDYN_LAUNCH_SWEEP(true, kSweep3);
    } else {
      PDYN_LAUNCH_SWEEP(false, kSweep1);
      PDYN_LAUNCH_SWEEP(false, kSweep2);
      if (MODE & kModeFD) PDYN_LAUNCH_SWEEP(false, kSweep3);
    }
#undef PDYN_LAUNCH_SWEEP
    if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
    return PDYN_OK;
  }
  if (m->n_chains == 1)
    hipLaunchKernelGGL((k_dynamics<T, MODE, true>), dim3(grid), dim3(block), 0, s, b->n_states,
                       m->n_links_max, lanes, table, wtable, q, qd, qdd_in, tau_in, tau_out, qdd_out,
                       static_cast<const T*>(b->tip_wrench), ba, scratch, status);
  else
    hipLaunchKernelGGL((k_dynamics<T, MODE, false>), dim3(grid), dim3(block), 0, s, b->n_states,
                       m->n_links_max, lanes, table, wtable, q, qd, qdd_in, tau_in, tau_out, qdd_out,
                       static_cast<const T*>(b->tip_wrench), ba, scratch, status);
  if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
  return PDYN_OK;
}

// Forward dynamics by JSIIA (FD) or the joint-space inertia alone, shared chain only.
template <class T, bool FD>
int run_jsiia(const pdyn_model* m, const pdyn_batch* b, const T* q, const T* qd, const T* tau, T* out, void* ws,
              size_t ws_bytes, void* stream) {
  const int op = FD ? PDYN_OP_JSIIA_FD : PDYN_OP_MASS_MATRIX;
  int st = check_model_batch(m, b);
  if (st) return st;
  if (m->n_chains != 1) return PDYN_EUNSUPPORTED;
  const pdyn_batch bt = tuned_batch(op, m, b, sizeof(T));
  b = &bt;
  if (b->n_states == 0) return PDYN_OK;
  if ((st = check_ptrs<T>({q, out}))) return st;
  if (FD && (st = check_ptrs<T>({qd, tau}))) return st;
  if ((st = check_ptrs<T>({m->placement, m->twist, m->inertia}))) return st;
  if (m->prepared && !aligned(m->prepared, kAlign)) return PDYN_EALIGN;
  if (b->tip_wrench && !aligned(b->tip_wrench, sizeof(T))) return PDYN_EALIGN;
  if (!ws) return PDYN_EINVAL;
  if (!aligned(ws, kAlign)) return PDYN_EALIGN;
  Layout L;
  if ((st = layout_for(op, m, b, sizeof(T), &L))) return st;
  if (ws_bytes < L.total) return PDYN_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned* status = static_cast<unsigned*>(ws);
  char* base = static_cast<char*>(ws) + kStatusBytes;
  const char* tbase = m->prepared ? static_cast<const char*>(m->prepared) : base;
  if (!m->prepared && (st = launch_link_table<T>(m, base, s))) return st;
  BoundaryArgs<T> ba;
  for (int k = 0; k < 6; ++k) { ba.V0[k] = (T)b->base_vel[k]; ba.dV0[k] = (T)b->base_acc[k]; }
  unsigned grid, block;
  launch_shape(b, &grid, &block);
  double* const work = reinterpret_cast<double*>(base + L.scratch_off);
  const int n = m->n_links_max;
  // forward dynamics up to 32 links: M and tau-hat here, the solve by a team of lanes per state
  const bool team = FD && n <= 32;
#define PDYN_LAUNCH_JSIIA(SOLVE)                                                                                   \
  hipLaunchKernelGGL((k_jsiia<T, FD, SOLVE>), dim3(grid), dim3(block), 0, s, b->n_states, n,                       \
                     reinterpret_cast<const T*>(tbase + L.table_off),                                              \
                     reinterpret_cast<const double*>(tbase + L.wtable_off), q, FD ? qd : nullptr,                  \
                     FD ? tau : nullptr, FD ? out : nullptr, FD ? nullptr : out,                                   \
                     static_cast<const T*>(b->tip_wrench), ba, work, status)
  if (team) PDYN_LAUNCH_JSIIA(false);
  else PDYN_LAUNCH_JSIIA(true);
#undef PDYN_LAUNCH_JSIIA
  if (team) {
    const int NT = n <= 8 ? 8 : (n <= 16 ? 16 : 32);
    const long lanes_total = (long)b->n_states * NT;
    const unsigned g = (unsigned)((lanes_total + 255) / 256);
    const size_t lds = (size_t)(256 / NT) * NT * NT * sizeof(double);
#define PDYN_LAUNCH_CHOL(NN)                                                                                       \
  do {                                                                                                             \
    if (lds > 65536 && hipFuncSetAttribute(reinterpret_cast<const void*>(&k_jsiia_chol<T, NN>),                    \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)    \
      return PDYN_ELAUNCH;                                                                                         \
    hipLaunchKernelGGL((k_jsiia_chol<T, NN>), dim3(g), dim3(256), lds, s, b->n_states, n, work, out, status);      \
  } while (0)
    switch (NT) {
      case 8: PDYN_LAUNCH_CHOL(8); break;
      case 16: PDYN_LAUNCH_CHOL(16); break;
      default: PDYN_LAUNCH_CHOL(32); break;
    }
#undef PDYN_LAUNCH_CHOL
  }
  if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
  return PDYN_OK;
}

// Second-derivative mode: the status word, then the link tables unless the model is prepared.
size_t hessian_ws_bytes(const pdyn_model* m, size_t scalar) {
  return kStatusBytes + (m->prepared ? 0 : tables_bytes(m, scalar, nullptr));
}

// Jacobian mode: the workspace holds the adjoint's workspace for one chunk of
// expanded rows (status word first), then the expanded q, qd, third input and
// cotangents ([rows][n] each) and tip wrenches ([rows][6]).
constexpr int64_t kJacRows = 1 << 17;  // rows (state x cotangent) per adjoint launch
struct JacLayout {
  int64_t chunk_states;
  size_t vjp_bytes, q_off, qd_off, x3_off, bar_off, tip_off, total;
};
int jac_layout(int vjp_op, const pdyn_model* m, const pdyn_batch* b, size_t scalar, JacLayout* J) {
  const int64_t n = m->n_links_max;
  J->chunk_states = std::max<int64_t>(1, std::min<int64_t>(b->n_states, kJacRows / n));
  pdyn_batch bc = *b;
  const int64_t rows = J->chunk_states * n;
  if (rows > INT32_MAX) return PDYN_EUNSUPPORTED;
  bc.n_states = (int32_t)rows;
  const pdyn_batch bt = tuned_batch(vjp_op, m, &bc, scalar);
  Layout L;
  const int st = layout_for(vjp_op, m, &bt, scalar, &L);
  if (st) return st;
  J->vjp_bytes = align_up(L.total);
  const size_t arr = align_up((size_t)rows * (size_t)n * scalar);
  J->q_off = J->vjp_bytes;
  J->qd_off = J->q_off + arr;
  J->x3_off = J->qd_off + arr;
  J->bar_off = J->x3_off + arr;
  J->tip_off = J->bar_off + arr;
  J->total = J->tip_off + align_up((size_t)rows * 6 * scalar);
  return PDYN_OK;
}

template <class T, int OP>
int run_vjp(const pdyn_model* m, const pdyn_batch* b, const T* q, const T* qd, const T* qdd, const T* bar_in,
            T* q_bar, T* qd_bar, T* out3, T* inertia_bar, void* ws, size_t ws_bytes, void* stream);

// Full Jacobians of a shared chain's ID (x3 = qdd; J3 = d tau / d qdd = M) or FD
// (x3 = qdd from FD; J3 = d qdd / d tau = M^-1), [n_states][n][n] each.
template <class T, int OP>
int run_jacobian(const pdyn_model* m, const pdyn_batch* b, const T* q, const T* qd, const T* x3, T* J1, T* J2,
                 T* J3, void* ws, size_t ws_bytes, void* stream) {
  const int vjp_op = OP == kVjpID ? PDYN_OP_RNEA_ID_VJP : PDYN_OP_ABA_FD_VJP;
  int st = check_model_batch(m, b);
  if (st) return st;
  if (m->n_chains != 1) return PDYN_EUNSUPPORTED;
  if (b->n_states == 0) return PDYN_OK;
  if ((st = check_ptrs<T>({q, qd, x3, J1, J2, J3}))) return st;
  if (b->tip_wrench && !aligned(b->tip_wrench, sizeof(T))) return PDYN_EALIGN;
  if (!ws) return PDYN_EINVAL;
  if (!aligned(ws, kAlign)) return PDYN_EALIGN;
  JacLayout jl;
  if ((st = jac_layout(vjp_op, m, b, sizeof(T), &jl))) return st;
  if (ws_bytes < jl.total) return PDYN_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* const base = static_cast<char*>(ws);
  T* const eq = reinterpret_cast<T*>(base + jl.q_off);
  T* const eqd = reinterpret_cast<T*>(base + jl.qd_off);
  T* const ex3 = reinterpret_cast<T*>(base + jl.x3_off);
  T* const ebar = reinterpret_cast<T*>(base + jl.bar_off);
  T* const etip = reinterpret_cast<T*>(base + jl.tip_off);
  const T* tip = static_cast<const T*>(b->tip_wrench);
  const int64_t n = m->n_links_max;
  for (int64_t s0 = 0; s0 < b->n_states; s0 += jl.chunk_states) {
    const int64_t ms = std::min<int64_t>(jl.chunk_states, b->n_states - s0);
    const int64_t rows = ms * n;
    const int64_t blocks = std::min<int64_t>((rows * n + 255) / 256, 8192);
    hipLaunchKernelGGL(k_jac_expand<T>, dim3((unsigned)blocks), dim3(256), 0, s, rows, (int)n, q + s0 * n,
                       qd + s0 * n, x3 + s0 * n, tip ? tip + s0 * 6 : nullptr, eq, eqd, ex3, ebar, etip);
    if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
    pdyn_batch bc = *b;
    bc.n_states = (int32_t)rows;
    bc.tip_wrench = tip ? etip : nullptr;
    const int64_t off = s0 * n * n;
    if ((st = run_vjp<T, OP>(m, &bc, eq, eqd, ex3, ebar, J1 + off, J2 + off, J3 + off, nullptr, ws, jl.vjp_bytes,
                             stream)))
      return st;
  }
  return PDYN_OK;
}

// Second derivatives of a shared chain's inverse dynamics: one thread per
// (state, requested block, j, k), the e1e2 parts of tau_0..tau_{n-1} going to
// H_b[s][i][j][k]. The (q, q) and (qd, qd) blocks are symmetric in (j, k): their
// threads take j <= k only and write both H[i][j][k] and H[i][k][j]. Within a
// block the threads run over rows j with k fastest, so for each i a wavefront
// writes consecutive words.
template <class T> struct HessOut {
  T* p[4];     // output of each requested block, in request order
  int blk[4];  // its block code (0 (q,q), 1 (q,qd), 2 (qd,qd), 3 (q,qdd))
  int nb;
};
PD_HD bool hess_symmetric(int block) { return block == 0 || block == 2; }
// Threads of one state: n(n+1)/2 for a symmetric block, n^2 otherwise.
template <class T> PD_HD int64_t hess_threads_per_state(const HessOut<T>& ho, int n) {
  int64_t per = 0;
  for (int b = 0; b < ho.nb; ++b) per += hess_symmetric(ho.blk[b]) ? (int64_t)n * (n + 1) / 2 : (int64_t)n * n;
  return per;
}

template <class T>
__global__ void __launch_bounds__(256) k_id_hessian(int64_t n_states, int n, const T* table, const T* q,
                                                    const T* qd, const T* qdd, BoundaryArgs<T> ba, const T* tip,
                                                    HessOut<T> ho, unsigned* status) {
  const int64_t nn = (int64_t)n * n, per = hess_threads_per_state(ho, n), total = n_states * per;
  const Sp<T> V0 = {v3(ba.V0[0], ba.V0[1], ba.V0[2]), v3(ba.V0[3], ba.V0[4], ba.V0[5])};
  const Sp<T> dV0 = {v3(ba.dV0[0], ba.dV0[1], ba.dV0[2]), v3(ba.dV0[3], ba.dV0[4], ba.dV0[5])};
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = t / per;
    int64_t r = t - s * per;
    int bi = 0;
    for (; bi < ho.nb - 1; ++bi) {
      const int64_t c = hess_symmetric(ho.blk[bi]) ? (int64_t)n * (n + 1) / 2 : nn;
      if (r < c) break;
      r -= c;
    }
    const bool sym = hess_symmetric(ho.blk[bi]);
    int j, k;
    if (sym) {  // row j holds k = j .. n-1
      j = 0;
      while (r >= n - j) {
        r -= n - j;
        ++j;
      }
      k = j + (int)r;
    } else {
      j = (int)(r / n);
      k = (int)(r - (int64_t)j * n);
    }
    Sp<T> F;
    if (tip) {
      const T* f = tip + 6 * s;
      F = {v3(f[0], f[1], f[2]), v3(f[3], f[4], f[5])};
    }
    T* const H = ho.p[bi] + s * nn * n;
    const int64_t jk = (int64_t)j * n + k, kj = (int64_t)k * n + j;
    bool finite = true;
    id_hessian_one<T>(n, table, q + s * n, qd + s * n, qdd + s * n, V0, dV0, tip ? &F : nullptr, ho.blk[bi], j, k,
                      [&](int i, T v) {
                        H[(int64_t)i * nn + jk] = v;
                        if (sym && j != k) H[(int64_t)i * nn + kj] = v;
                        finite = finite && isfinite(v);
                      });
    if (!finite) atomicOr(status, PDYN_STATUS_NONFINITE);
  }
}

template <class T>
int run_id_hessian(const pdyn_model* m, const pdyn_batch* b, const T* q, const T* qd, const T* qdd, T* H_qq,
                   T* H_qqd, T* H_qdqd, T* H_qqdd, void* ws, size_t ws_bytes, void* stream) {
  int st = check_model_batch(m, b);
  if (st) return st;
  if (m->n_chains != 1) return PDYN_EUNSUPPORTED;
  HessOut<T> ho{};
  T* const outs[4] = {H_qq, H_qqd, H_qdqd, H_qqdd};
  for (int k = 0; k < 4; ++k)
    if (outs[k]) {
      if (!aligned(outs[k], sizeof(T))) return PDYN_EALIGN;
      ho.p[ho.nb] = outs[k];
      ho.blk[ho.nb++] = k;
    }
  if (ho.nb == 0) return PDYN_EINVAL;
  if (b->n_states == 0) return PDYN_OK;
  if ((st = check_ptrs<T>({q, qd, qdd, m->placement, m->twist, m->inertia}))) return st;
  if (b->tip_wrench && !aligned(b->tip_wrench, sizeof(T))) return PDYN_EALIGN;
  if (m->prepared && !aligned(m->prepared, kAlign)) return PDYN_EALIGN;
  if (!ws) return PDYN_EINVAL;
  if (!aligned(ws, kAlign)) return PDYN_EALIGN;
  if (ws_bytes < hessian_ws_bytes(m, sizeof(T))) return PDYN_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned* status = static_cast<unsigned*>(ws);
  char* base = static_cast<char*>(ws) + kStatusBytes;
  const char* tbase = m->prepared ? static_cast<const char*>(m->prepared) : base;
  if (!m->prepared && (st = launch_link_table<T>(m, base, s))) return st;
  BoundaryArgs<T> ba;
  for (int k = 0; k < 6; ++k) { ba.V0[k] = (T)b->base_vel[k]; ba.dV0[k] = (T)b->base_acc[k]; }
  const int64_t n = m->n_links_max;
  const int64_t total = (int64_t)b->n_states * hess_threads_per_state(ho, (int)n);
  const int64_t grid = std::min<int64_t>((total + 255) / 256, int64_t(1) << 16);
  hipLaunchKernelGGL(k_id_hessian<T>, dim3((unsigned)grid), dim3(256), 0, s, (int64_t)b->n_states, (int)n,
                     reinterpret_cast<const T*>(tbase), q, qd, qdd, ba, static_cast<const T*>(b->tip_wrench), ho,
                     status);
  if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
  return PDYN_OK;
}

// Articulated-body inertias Jhat_i (eq. (7)) of a shared chain by the associative
// scan of abi_scan.hpp: a team of P lanes per state (P a power of two, 1..128)
// in workgroups of max(64, P) threads (64 / P states each, or one state whose
// team spans P / 64 wavefronts). P = 1 is the serial recursion, one lane per
// state. With P > 1 the lanes of a team fold their segments, combine the
// aggregates by a Kogge-Stone suffix scan through LDS ([kAbiElWords][workgroup]
// doubles, one slot per lane, workgroup barriers between the steps) and rerun
// their segments from the carry. Jhat is written whole, [n_states][n][6][6].
template <class T, bool SCAN, int BT>  // BT = workgroup threads, max(64, P)
__global__ void __launch_bounds__(BT) k_abi_scan(int n_states, int n, int P, const T* __restrict__ table,
                                                 const double* __restrict__ wtable, const T* q, T* Jhat,
                                                 unsigned* status) {
  extern __shared__ double abi_lds[];
  const int lane = threadIdx.x;  // BT / P teams, or one team of P lanes over P / 64 wavefronts
  const int k = lane & (P - 1);
  const int64_t s = (int64_t)blockIdx.x * (BT / P) + lane / P;
  const bool active = s < n_states;
  const T* qs = q + (active ? s : 0) * n;
  const Seg g = active ? segment_of(n, P, k) : Seg{0, 0};
  const AbiPoses<T, const T*, const double*> poses{table, wtable, qs};
  bool ok = true;
  Sym6<double> carry{};
  bool has_carry = false;
  if (SCAN) {
    abi_store(abi_lds, BT, lane, abi_fold_segment(n, g.a, g.b, wtable, poses, &ok));
    for (int d = 1; d < P; d <<= 1) {
      __syncthreads();
      const bool upd = k + d < P;
      AbiEl r;
      if (upd) r = abi_compose(AbiView{abi_lds, BT, lane}, AbiView{abi_lds, BT, lane + d}, &ok);
      __syncthreads();
      if (upd) abi_store(abi_lds, BT, lane, r);
    }
    __syncthreads();
    has_carry = k + 1 < P && !AbiView{abi_lds, BT, lane + 1}.ident();
    if (has_carry) carry = AbiView{abi_lds, BT, lane + 1}.Q();
  }
  bool finite = true;
  T* const out = Jhat + (active ? s : 0) * n * 36;
  abi_serial_segment(n, g.a, g.b, wtable, poses, carry,
                     [&](int i, const Sym6<double>& J) {
                       const M6 m = m6_of(J);
                       T* o = out + (int64_t)i * 36;
#pragma unroll
                       for (int e = 0; e < 36; ++e) {
                         const T v = (T)m.m[e];
                         o[e] = v;
                         finite = finite && __builtin_isfinite(v);
                       }
                     },
                     &ok);
  const unsigned bits = (finite ? 0u : kStatusNonFinite) | (ok ? 0u : kStatusPivot);
  if (active && bits) __hip_atomic_fetch_or(status, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workspace of the articulated-inertia scan: the status word, then the link tables unless prepared.
size_t abi_scan_ws_bytes(const pdyn_model* m, size_t scalar) {
  return kStatusBytes + (m->prepared ? 0 : tables_bytes(m, scalar, nullptr));
}

// Lanes per state of the scans: the batch's `segments`, or by default the
// smallest power of two that gives the batch `target` lanes, at most 64 and
// at least 4 links per segment. The articulated inertias alone take 16384
// lanes (one wavefront per compute unit); the scanned forward dynamics,
// whose serial phases hold four recursions, pays for twice as many (measured
// best at 32 x 16384, 128 x 1024 (4 links per segment), 512 x 256 and
// 1024 x 64 links x states).
int abi_scan_lanes(const pdyn_model* m, const pdyn_batch* b, int64_t target = 16384) {
  if (b->segments > 0) return b->segments;
  int P = 1;
  while (P < kMaxScanLanes && (int64_t)b->n_states * P < target && m->n_links_max >= 8 * P) P *= 2;
  return P;
}

// The scans take `segments` up to kMaxScanLanes (a power of two; 0 = default);
// the rest of the batch is checked as for every call.
int check_scan_batch(const pdyn_model* m, const pdyn_batch* b) {
  if (!b) return PDYN_EINVAL;
  pdyn_batch c = *b;
  c.segments = 0;
  const int st = check_model_batch(m, &c);
  if (st) return st;
  if (b->segments < 0 || b->segments > kMaxScanLanes || (b->segments & (b->segments - 1))) return PDYN_EINVAL;
  return PDYN_OK;
}

// Workgroup threads and dynamic LDS of a scan launch with P lanes per state.
unsigned scan_block(int P) { return P > 64 ? (unsigned)P : 64u; }
size_t scan_lds(int P) { return (size_t)kAbiElWords * scan_block(P) * sizeof(double); }

template <class T>
int run_abi_scan(const pdyn_model* m, const pdyn_batch* b, const T* q, T* Jhat, void* ws, size_t ws_bytes,
                 void* stream) {
  int st = check_scan_batch(m, b);
  if (st) return st;
  if (m->n_chains != 1) return PDYN_EUNSUPPORTED;
  if (b->n_states == 0) return PDYN_OK;
  if ((st = check_ptrs<T>({q, Jhat, m->placement, m->twist, m->inertia}))) return st;
  if (m->prepared && !aligned(m->prepared, kAlign)) return PDYN_EALIGN;
  if (!ws) return PDYN_EINVAL;
  if (!aligned(ws, kAlign)) return PDYN_EALIGN;
  if (ws_bytes < abi_scan_ws_bytes(m, sizeof(T))) return PDYN_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned* status = static_cast<unsigned*>(ws);
  char* base = static_cast<char*>(ws) + kStatusBytes;
  const char* tbase = m->prepared ? static_cast<const char*>(m->prepared) : base;
  if (!m->prepared && (st = launch_link_table<T>(m, base, s))) return st;
  size_t woff;
  tables_bytes(m, sizeof(T), &woff);
  const int P = abi_scan_lanes(m, b);
  const unsigned block = scan_block(P);
  const int64_t per_block = block / P;
  const int64_t grid = ((int64_t)b->n_states + per_block - 1) / per_block;
  const size_t lds = scan_lds(P);
  const T* const tab = reinterpret_cast<const T*>(tbase);
  const double* const wtab = reinterpret_cast<const double*>(tbase + woff);
  if (P > 64) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(&k_abi_scan<T, true, kMaxScanLanes>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
      return PDYN_ELAUNCH;
    hipLaunchKernelGGL((k_abi_scan<T, true, kMaxScanLanes>), dim3((unsigned)grid), dim3(block), lds, s,
                       b->n_states, (int)m->n_links_max, P, tab, wtab, q, Jhat, status);
  } else if (P > 1)
    hipLaunchKernelGGL((k_abi_scan<T, true, 64>), dim3((unsigned)grid), dim3(block), lds, s, b->n_states,
                       (int)m->n_links_max, P, tab, wtab, q, Jhat, status);
  else
    hipLaunchKernelGGL((k_abi_scan<T, false, 64>), dim3((unsigned)grid), dim3(64), 0, s, b->n_states,
                       (int)m->n_links_max, 1, tab, wtab, q, Jhat, status);
  if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
  return PDYN_OK;
}

// Forward dynamics of a shared chain with every recursion scanned (fd_scan.hpp):
// a team of P lanes per state in workgroups as in k_abi_scan, four phases of
// fold, Kogge-Stone scan through LDS ([85 words][workgroup] doubles, reused by
// every phase) and apply; SPLIT runs the third phase as two scans (the bias
// wrench, then z-hat) instead of one scan of the merged recursion. Per-link values (Fhat, U, 1/D, c-hat, the link transform) in `scratch`,
// [n_states][n][kFdScanWords] doubles; a lane touches only its own links there,
// so the phases need no ordering beyond the workgroup barriers around the LDS
// exchanges.
// Kogge-Stone inclusive scan of the affine elements that every lane of the
// workgroup has stored in LDS ([word][BT]): suffix (lane k takes x_k o x_{k+d})
// or prefix (x_k o x_{k-d}) within each team of P lanes; ends with a barrier.
template <int BT, bool SUFFIX>
__device__ __forceinline__ void lds_aff_scan(double* lds, int lane, int k, int P) {
  for (int d = 1; d < P; d <<= 1) {
    __syncthreads();
    const bool upd = SUFFIX ? k + d < P : k >= d;
    AffEl r;
    if (upd) r = aff_compose(aff_load(lds, BT, lane), aff_load(lds, BT, SUFFIX ? lane + d : lane - d));
    __syncthreads();
    if (upd) aff_store(lds, BT, lane, r);
  }
  __syncthreads();
}

template <class T, int BT, bool SPLIT>  // BT = workgroup threads, max(64, P), as in k_abi_scan; SPLIT: phase 3
__global__ void __launch_bounds__(BT) k_fd_scan(int n_states, int n, int P, const T* __restrict__ table,
                                                const double* __restrict__ wtable, const T* q, const T* qd,
                                                const T* tau, T* qdd, const T* tip, BoundaryArgs<T> ba,
                                                double* scratch, unsigned* status) {
  extern __shared__ double fs_lds[];
  const int lane = threadIdx.x;
  const int k = lane & (P - 1);
  const int64_t s = (int64_t)blockIdx.x * (BT / P) + lane / P;
  const bool active = s < n_states;
  const int64_t so = active ? s : 0;
  const T* const qs = q + so * n;
  const T* const qds = qd + so * n;
  const T* const taus = tau + so * n;
  const Seg g = active ? segment_of(n, P, k) : Seg{0, 0};
  const FdScanScr scr{scratch + so * n * kFdScanWords};
  const FdPoses<T, const T*, const double*> poses{g, table, wtable, qs, scr};
  const Sp<double> V0 = {v3((double)ba.V0[0], (double)ba.V0[1], (double)ba.V0[2]),
                         v3((double)ba.V0[3], (double)ba.V0[4], (double)ba.V0[5])};
  const Sp<double> dV0 = {v3((double)ba.dV0[0], (double)ba.dV0[1], (double)ba.dV0[2]),
                          v3((double)ba.dV0[3], (double)ba.dV0[4], (double)ba.dV0[5])};
  Sp<double> Ftip = sp_zero<double>();
  if (tip) {
    const T* f = tip + 6 * so;
    Ftip = {v3((double)f[0], (double)f[1], (double)f[2]), v3((double)f[3], (double)f[4], (double)f[5])};
  }
  bool ok = true;
  // 1: velocities and bias accelerations (inclusive prefix), then Fhat
  fwd_store(fs_lds, BT, lane, fds_bias_fold<T>(g, table, wtable, qs, qds, V0, dV0, scr));
  for (int d = 1; d < P; d <<= 1) {
    __syncthreads();
    const bool upd = k >= d;
    FwdOp<double> r;
    if (upd) r = fwd_combine(fwd_load(fs_lds, BT, lane), fwd_load(fs_lds, BT, lane - d));
    __syncthreads();
    if (upd) fwd_store(fs_lds, BT, lane, r);
  }
  __syncthreads();
  Sp<double> dV = dV0, V = V0;
  if (k > 0) {
    const FwdOp<double> e = fwd_load(fs_lds, BT, lane - 1);
    dV = e.x1;
    V = e.x2;
  }
  __syncthreads();
  fds_bias_apply<T>(g, wtable, qds, dV, V, scr);
  // 2: articulated inertias (inclusive suffix), then U and 1/D
  abi_store(fs_lds, BT, lane, abi_fold_segment(n, g.a, g.b, wtable, poses, &ok));
  for (int d = 1; d < P; d <<= 1) {
    __syncthreads();
    const bool upd = k + d < P;
    AbiEl r;
    if (upd) r = abi_compose(AbiView{fs_lds, BT, lane}, AbiView{fs_lds, BT, lane + d}, &ok);
    __syncthreads();
    if (upd) abi_store(fs_lds, BT, lane, r);
  }
  __syncthreads();
  Sym6<double> carry{};
  if (k + 1 < P && !AbiView{fs_lds, BT, lane + 1}.ident()) carry = AbiView{fs_lds, BT, lane + 1}.Q();
  __syncthreads();
  fds_abi_apply(n, g, wtable, poses, carry, scr, &ok);
  // 3: bias wrench and z-hat (inclusive suffix), then c-hat: one scan of the merged recursion, or
  // (SPLIT) the bias wrench and then z-hat as two scans
  if (SPLIT) {
    aff_store(fs_lds, BT, lane, fds_f_fold(n, g, wtable, poses, scr));
    lds_aff_scan<BT, true>(fs_lds, lane, k, P);
    Sp<double> Fc = Ftip;
    if (k + 1 < P) {
      const AffEl e = aff_load(fs_lds, BT, lane + 1);
      Fc = m6_apply(e.M, Ftip) + sp_of(e.c);
    }
    __syncthreads();
    fds_f_apply<T>(n, g, wtable, poses, taus, Fc, scr);
    aff_store(fs_lds, BT, lane, fds_zs_fold(n, g, wtable, poses, scr));
    lds_aff_scan<BT, true>(fs_lds, lane, k, P);
    const Sp<double> Zc = k + 1 < P ? aff_load_c(fs_lds, BT, lane + 1) : sp_zero<double>();
    __syncthreads();
    fds_zs_apply(n, g, wtable, poses, Zc, scr);
  } else {
    aff_store(fs_lds, BT, lane, fds_z_fold<T>(n, g, wtable, poses, taus, scr));
    lds_aff_scan<BT, true>(fs_lds, lane, k, P);
    Sp<double> Pc = Ftip;
    if (k + 1 < P) {
      const AffEl e = aff_load(fs_lds, BT, lane + 1);
      Pc = m6_apply(e.M, Ftip) + sp_of(e.c);
    }
    __syncthreads();
    fds_z_apply<T>(n, g, wtable, poses, taus, Pc, scr);
  }
  // 4: lambda (inclusive prefix), then qdd
  aff_store(fs_lds, BT, lane, fds_l_fold(g, wtable, scr));
  lds_aff_scan<BT, false>(fs_lds, lane, k, P);
  const Sp<double> lam = k > 0 ? aff_load_c(fs_lds, BT, lane - 1) : sp_zero<double>();
  bool finite = true;
  T* const out = qdd + so * n;
  fds_l_apply(g, wtable, lam, scr, [&](int i, double v) {
    const T x = (T)v;
    out[i] = x;
    finite = finite && __builtin_isfinite(x);
  });
  const unsigned bits = (finite ? 0u : kStatusNonFinite) | (ok ? 0u : kStatusPivot);
  if (active && bits) __hip_atomic_fetch_or(status, bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workspace of the scanned forward dynamics: the status word, the link tables
// unless prepared, then the per-link scratch, [n_states][n][kFdScanWords] doubles.
size_t fd_scan_ws_bytes(const pdyn_model* m, const pdyn_batch* b, size_t scalar, size_t* scratch_off) {
  const size_t t = kStatusBytes + (m->prepared ? 0 : align_up(tables_bytes(m, scalar, nullptr)));
  if (scratch_off) *scratch_off = t;
  return t + align_up((size_t)b->n_states * (size_t)m->n_links_max * kFdScanWords * sizeof(double));
}

template <class T>
int run_fd_scan(const pdyn_model* m, const pdyn_batch* b, const T* q, const T* qd, const T* tau, T* qdd, void* ws,
                size_t ws_bytes, void* stream) {
  int st = check_scan_batch(m, b);
  if (st) return st;
  if (b->variant != 0 && b->variant != 1 && b->variant != 2) return PDYN_EINVAL;
  if (m->n_chains != 1) return PDYN_EUNSUPPORTED;
  if (b->n_states == 0) return PDYN_OK;
  if ((st = check_ptrs<T>({q, qd, tau, qdd, m->placement, m->twist, m->inertia}))) return st;
  if (b->tip_wrench && !aligned(b->tip_wrench, sizeof(T))) return PDYN_EALIGN;
  if (m->prepared && !aligned(m->prepared, kAlign)) return PDYN_EALIGN;
  if (!ws) return PDYN_EINVAL;
  if (!aligned(ws, kAlign)) return PDYN_EALIGN;
  size_t scratch_off;
  if (ws_bytes < fd_scan_ws_bytes(m, b, sizeof(T), &scratch_off)) return PDYN_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned* status = static_cast<unsigned*>(ws);
  char* base = static_cast<char*>(ws) + kStatusBytes;
  const char* tbase = m->prepared ? static_cast<const char*>(m->prepared) : base;
  if (!m->prepared && (st = launch_link_table<T>(m, base, s))) return st;
  size_t woff;
  tables_bytes(m, sizeof(T), &woff);
  BoundaryArgs<T> ba;
  for (int k = 0; k < 6; ++k) { ba.V0[k] = (T)b->base_vel[k]; ba.dV0[k] = (T)b->base_acc[k]; }
  const int P = abi_scan_lanes(m, b, 32768);
  const unsigned block = scan_block(P);
  const int64_t per_block = block / P;
  const int64_t grid = ((int64_t)b->n_states + per_block - 1) / per_block;
  const size_t lds = scan_lds(P);
  const bool split = b->variant == 2;
  if (P > 64 &&
      hipFuncSetAttribute(split ? reinterpret_cast<const void*>(&k_fd_scan<T, kMaxScanLanes, true>)
                                : reinterpret_cast<const void*>(&k_fd_scan<T, kMaxScanLanes, false>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return PDYN_ELAUNCH;
  const T* const tab = reinterpret_cast<const T*>(tbase);
  const double* const wtab = reinterpret_cast<const double*>(tbase + woff);
  const T* const tip = static_cast<const T*>(b->tip_wrench);
  double* const scratch = reinterpret_cast<double*>(static_cast<char*>(ws) + scratch_off);
#define PDYN_LAUNCH_FD_SCAN(BT, SPLIT)                                                                          \
  hipLaunchKernelGGL((k_fd_scan<T, BT, SPLIT>), dim3((unsigned)grid), dim3(block), lds, s, b->n_states,          \
                     (int)m->n_links_max, P, tab, wtab, q, qd, tau, qdd, tip, ba, scratch, status)
  if (P > 64 && split) PDYN_LAUNCH_FD_SCAN(kMaxScanLanes, true);
  else if (P > 64) PDYN_LAUNCH_FD_SCAN(kMaxScanLanes, false);
  else if (split) PDYN_LAUNCH_FD_SCAN(64, true);
  else PDYN_LAUNCH_FD_SCAN(64, false);
#undef PDYN_LAUNCH_FD_SCAN
  if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
  return PDYN_OK;
}

size_t rollout_layout(int with_grad, const pdyn_model* m, const pdyn_batch* b, int every, size_t scalar,
                      size_t* scratch_off, size_t* rows_off, size_t* acc_off) {
  size_t woff;
  const size_t tb = tables_bytes(m, scalar, &woff);
  const size_t nm = (size_t)m->n_links_max, B = (size_t)b->n_states;
  size_t off = m->prepared ? 0 : tb;
  *scratch_off = off;
  if (!with_grad) {
    off += align_up(nm * (size_t)ScratchWords<kModeFD>::value * B * scalar);
    *rows_off = *acc_off = off;
    return off + kStatusBytes;
  }
  off += align_up(nm * (size_t)kVjpWords * B * scalar);
  *rows_off = off;
  off += align_up(B * (size_t)(3 * every + 6) * nm * scalar);
  *acc_off = off;
  off += align_up(nm * 10 * B * scalar);
  return off + kStatusBytes;
}

template <class T>
int check_rollout_args(const pdyn_model* m, const pdyn_batch* b, int steps, double dt, int every) {
  int st = check_model_batch(m, b);
  if (st) return st;
  if (steps < 0 || every < 1 || !(dt == dt)) return PDYN_EINVAL;
  if (b->tip_wrench) return PDYN_EUNSUPPORTED;  // rollouts run without an external tip wrench
  if ((st = check_ptrs<T>({m->placement, m->twist, m->inertia}))) return st;
  if (m->prepared && !aligned(m->prepared, kAlign)) return PDYN_EALIGN;
  return PDYN_OK;
}

template <class T>
int run_rollout(const pdyn_model* m, const pdyn_batch* b, int steps, double dt, int every, const T* tau_seq, T* q,
                T* qd, T* ckpt_q, T* ckpt_qd, void* ws, size_t ws_bytes, void* stream) {
  int st = check_rollout_args<T>(m, b, steps, dt, every);
  if (st) return st;
  if (b->n_states == 0 || steps == 0) return PDYN_OK;
  if ((st = check_ptrs<T>({tau_seq, q, qd, ckpt_q, ckpt_qd}))) return st;
  if (!ws) return PDYN_EINVAL;
  if (!aligned(ws, kAlign)) return PDYN_EALIGN;
  size_t so, ro, ao;
  if (ws_bytes < rollout_layout(0, m, b, every, sizeof(T), &so, &ro, &ao)) return PDYN_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned* status = static_cast<unsigned*>(ws);  // the first kStatusBytes of every workspace
  char* base = static_cast<char*>(ws) + kStatusBytes;
  size_t woff;
  tables_bytes(m, sizeof(T), &woff);
  const char* tbase = m->prepared ? static_cast<const char*>(m->prepared) : base;
  const LaneChain* const lanes = lane_map(m, tbase, sizeof(T));
  if (!m->prepared && (st = launch_link_table<T>(m, base, s))) return st;
  BoundaryArgs<T> ba;
  for (int k = 0; k < 6; ++k) { ba.V0[k] = (T)b->base_vel[k]; ba.dV0[k] = (T)b->base_acc[k]; }
  const long dofs = (m->n_chains == 1) ? (long)b->n_states * m->n_links_max : (long)m->n_links_total;
  unsigned grid, block;
  launch_shape(b, &grid, &block);
#define PDYN_LAUNCH_ROLLOUT(SH)                                                                                  \
  hipLaunchKernelGGL((k_rollout<T, SH>), dim3(grid), dim3(block), 0, s, b->n_states, m->n_links_max, lanes,         \
                     reinterpret_cast<const T*>(tbase),                                    \
                     reinterpret_cast<const double*>(tbase + woff), steps, (T)dt, every, tau_seq, q, qd, ckpt_q,   \
                     ckpt_qd, dofs, ba, reinterpret_cast<T*>(base + so), status)
  if (m->n_chains == 1)
    PDYN_LAUNCH_ROLLOUT(true);
  else
    PDYN_LAUNCH_ROLLOUT(false);
#undef PDYN_LAUNCH_ROLLOUT
  if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
  return PDYN_OK;
}

template <class T>
int run_rollout_vjp(const pdyn_model* m, const pdyn_batch* b, int steps, double dt, int every, const T* tau_seq,
                    const T* ckpt_q, const T* ckpt_qd, const T* qT_bar, const T* qdT_bar, T* q0_bar, T* qd0_bar,
                    T* tau_bar_seq, T* inertia_bar, void* ws, size_t ws_bytes, void* stream) {
  int st = check_rollout_args<T>(m, b, steps, dt, every);
  if (st) return st;
  if (b->n_states == 0) return PDYN_OK;
  if ((st = check_ptrs<T>({tau_seq, ckpt_q, ckpt_qd, qT_bar, qdT_bar, q0_bar, qd0_bar, tau_bar_seq}))) return st;
  if (inertia_bar && !aligned(inertia_bar, sizeof(T))) return PDYN_EALIGN;
  if (!ws) return PDYN_EINVAL;
  if (!aligned(ws, kAlign)) return PDYN_EALIGN;
  size_t so, ro, ao;
  if (ws_bytes < rollout_layout(1, m, b, every, sizeof(T), &so, &ro, &ao)) return PDYN_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned* status = static_cast<unsigned*>(ws);  // the first kStatusBytes of every workspace
  char* base = static_cast<char*>(ws) + kStatusBytes;
  size_t woff;
  tables_bytes(m, sizeof(T), &woff);
  const char* tbase = m->prepared ? static_cast<const char*>(m->prepared) : base;
  const LaneChain* const lanes = lane_map(m, tbase, sizeof(T));
  if (!m->prepared && (st = launch_link_table<T>(m, base, s))) return st;
  BoundaryArgs<T> ba;
  for (int k = 0; k < 6; ++k) { ba.V0[k] = (T)b->base_vel[k]; ba.dV0[k] = (T)b->base_acc[k]; }
  const long dofs = (m->n_chains == 1) ? (long)b->n_states * m->n_links_max : (long)m->n_links_total;
  const unsigned grid = (unsigned)((b->n_states + kBlock - 1) / kBlock);
  T* acc = reinterpret_cast<T*>(base + ao);
#define PDYN_LAUNCH_RVJP(PI, SH)                                                                                 \
  hipLaunchKernelGGL((k_rollout_vjp<T, PI, SH>), dim3(grid), dim3(kBlock), 0, s, b->n_states,          \
                     m->n_links_max, lanes, reinterpret_cast<const T*>(tbase),                   \
                     reinterpret_cast<const double*>(tbase + woff), steps, (T)dt, every, tau_seq, ckpt_q,          \
                     ckpt_qd, qT_bar, qdT_bar, q0_bar, qd0_bar, tau_bar_seq, inertia_bar, dofs, ba,               \
                     reinterpret_cast<T*>(base + so), reinterpret_cast<T*>(base + ro), acc, status)
  if (!inertia_bar) {
    if (m->n_chains == 1)
      PDYN_LAUNCH_RVJP(kPiNone, true);
    else
      PDYN_LAUNCH_RVJP(kPiNone, false);
  } else if (m->n_chains == 1) {
    PDYN_LAUNCH_RVJP(kPiLanes, true);
    hipLaunchKernelGGL(k_reduce_lanes<T>, dim3(m->n_links_max * 10), dim3(256), 0, s, b->n_states, acc, inertia_bar);
  } else {
    PDYN_LAUNCH_RVJP(kPiDirect, false);
  }
#undef PDYN_LAUNCH_RVJP
  if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
  return PDYN_OK;
}

template <class T, int OP>
int run_vjp(const pdyn_model* m, const pdyn_batch* b, const T* q, const T* qd, const T* qdd, const T* bar_in,
            T* q_bar, T* qd_bar, T* out3, T* inertia_bar, void* ws, size_t ws_bytes, void* stream) {
  const int op = (OP == kVjpID) ? PDYN_OP_RNEA_ID_VJP : PDYN_OP_ABA_FD_VJP;
  int st = check_model_batch(m, b);
  if (st) return st;
  const pdyn_batch bt = tuned_batch(op, m, b, sizeof(T));
  b = &bt;
  if (b->n_states == 0) return PDYN_OK;
  if ((st = check_ptrs<T>({q, qd, qdd, bar_in, q_bar, qd_bar, out3}))) return st;
  if ((st = check_ptrs<T>({m->placement, m->twist, m->inertia}))) return st;
  if (inertia_bar && !aligned(inertia_bar, sizeof(T))) return PDYN_EALIGN;
  if (m->prepared && !aligned(m->prepared, kAlign)) return PDYN_EALIGN;
  if (b->tip_wrench && !aligned(b->tip_wrench, sizeof(T))) return PDYN_EALIGN;
  if (!ws) return PDYN_EINVAL;
  if (!aligned(ws, kAlign)) return PDYN_EALIGN;
  Layout L;
  if ((st = layout_for(op, m, b, sizeof(T), &L))) return st;
  if (ws_bytes < L.total) return PDYN_EWORKSPACE;

  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned* status = static_cast<unsigned*>(ws);  // the first kStatusBytes of every workspace
  char* base = static_cast<char*>(ws) + kStatusBytes;
  T* scratch = reinterpret_cast<T*>(base + L.scratch_off);
  T* partials = reinterpret_cast<T*>(base + L.partial_off);
  const char* tbase = m->prepared ? static_cast<const char*>(m->prepared) : base;
  const LaneChain* const lanes = lane_map(m, tbase, sizeof(T));
  const T* table = reinterpret_cast<const T*>(tbase + L.table_off);
  const double* wtable = reinterpret_cast<const double*>(tbase + L.wtable_off);
  if (!m->prepared) {
    if ((st = launch_link_table<T>(m, base, s))) return st;
  }
  BoundaryArgs<T> ba;
  for (int k = 0; k < 6; ++k) { ba.V0[k] = (T)b->base_vel[k]; ba.dV0[k] = (T)b->base_acc[k]; }
  const unsigned grid = (unsigned)((b->n_states + kBlock - 1) / kBlock);
  T* qdd_bar = (OP == kVjpID) ? out3 : nullptr;
  T* tau_bar = (OP == kVjpFD) ? out3 : nullptr;
  const T* tip = static_cast<const T*>(b->tip_wrench);
  const int vjp_variant = pick_variant(b, false);
  const bool split = vjp_variant == 2;
  const unsigned grid64 = (unsigned)((b->n_states + 63) / 64);
  T* xscratch = reinterpret_cast<T*>(base + L.xscratch_off);
  if (vjp_variant == 3) {  // the plain form: one launch per pass
#define PDYN_LAUNCH_VJP_PASS(PI, SH, PASS, PIOUT)                                                              \
  hipLaunchKernelGGL((k_vjp_pass<T, OP, PI, SH, PASS>), dim3(grid64), dim3(64), 0, s, b->n_states,              \
                     m->n_links_max, lanes, table, wtable, q, qd, qdd, bar_in, q_bar, qd_bar, qdd_bar, tau_bar, \
                     PIOUT, tip, ba, scratch, xscratch, status)
#define PDYN_LAUNCH_VJP_PASSES(PI, SH, PIOUT)                                                                  \
  do {                                                                                                         \
    PDYN_LAUNCH_VJP_PASS(PI, SH, kVjpPassX, PIOUT);                                                            \
    PDYN_LAUNCH_VJP_PASS(PI, SH, kVjpPassNeFwd, PIOUT);                                                        \
    PDYN_LAUNCH_VJP_PASS(PI, SH, kVjpPassWrench, PIOUT);                                                       \
    if (PI != kPiNone) PDYN_LAUNCH_VJP_PASS(PI, SH, kVjpPassInertia, PIOUT);                                   \
    PDYN_LAUNCH_VJP_PASS(PI, SH, kVjpPassBack, PIOUT);                                                         \
  } while (0)
    if (!inertia_bar) {
      if (m->n_chains == 1)
        PDYN_LAUNCH_VJP_PASSES(kPiNone, true, static_cast<T*>(nullptr));
      else
        PDYN_LAUNCH_VJP_PASSES(kPiNone, false, static_cast<T*>(nullptr));
    } else if (m->n_chains == 1) {
      PDYN_LAUNCH_VJP_PASSES(kPiLanes, true, partials);
      hipLaunchKernelGGL(k_reduce_lanes<T>, dim3(m->n_links_max * 10), dim3(256), 0, s, b->n_states, partials,
                         inertia_bar);
    } else {
      PDYN_LAUNCH_VJP_PASSES(kPiDirect, false, inertia_bar);
    }
#undef PDYN_LAUNCH_VJP_PASSES
#undef PDYN_LAUNCH_VJP_PASS
    if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
    return PDYN_OK;
  }
  // ID adjoint: the wrenches of every link in LDS, after the transform ring; FD adjoint: the
  // articulated terms of every link (third wavefront)
  const size_t lds1 = OP == kVjpID
                          ? ((size_t)kPoseSlots * kPoseWordsF + (size_t)m->n_links_max * 6) * 64 * sizeof(T)
                          : ((size_t)m->n_links_max * kAbiWords + (size_t)kPoseSlots * kPoseWordsB) * 64 * sizeof(T);
  const size_t lds2 = lds1 + (size_t)kPoseSlots * kBackWords * 64 * sizeof(T);  // and the cut sweep's ring
  const int ovl = lds2 <= max_lds_bytes() ? 2 : (lds1 <= max_lds_bytes() ? 1 : 0);
  const size_t lds = ovl == 2 ? lds2 : lds1;
  const unsigned vjp_block = ((OP == kVjpFD && ovl >= 1) || ovl == 2) ? 256 : 128;
#define PDYN_LAUNCH_VJP_SPLIT(PI, SH, OV, PIOUT)                                                              \
  do {                                                                                                        \
    if (OV && lds > 65536 &&                                                                                  \
        hipFuncSetAttribute(reinterpret_cast<const void*>(&k_vjp_split<T, OP, PI, SH, OV>),                   \
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)              \
      return PDYN_ELAUNCH;                                                                                    \
    hipLaunchKernelGGL((k_vjp_split<T, OP, PI, SH, OV>), dim3(grid64), dim3(OV ? vjp_block : 128), OV ? lds : 0, s, \
                       b->n_states, m->n_links_max, lanes, table, wtable, q, qd, qdd, bar_in,   \
                       q_bar, qd_bar, qdd_bar, tau_bar, PIOUT, tip, ba, scratch, xscratch, status);           \
  } while (0)
#define PDYN_LAUNCH_VJP(PI, SH, PIOUT)                                                                        \
  do {                                                                                                        \
    if (split && ovl == 2)                                                                                    \
      PDYN_LAUNCH_VJP_SPLIT(PI, SH, 2, PIOUT);                                                                \
    else if (split && ovl == 1)                                                                               \
      PDYN_LAUNCH_VJP_SPLIT(PI, SH, 1, PIOUT);                                                                \
    else if (split)                                                                                           \
      PDYN_LAUNCH_VJP_SPLIT(PI, SH, 0, PIOUT);                                                                \
    else                                                                                                      \
      hipLaunchKernelGGL((k_vjp<T, OP, PI, SH>), dim3(grid), dim3(kBlock), 0, s, b->n_states,    \
                         m->n_links_max, lanes, table, wtable, q, qd, qdd, bar_in, q_bar, qd_bar, \
                         qdd_bar, tau_bar, PIOUT, tip, ba, scratch, status);                                  \
  } while (0)
  if (!inertia_bar) {
    if (m->n_chains == 1)
      PDYN_LAUNCH_VJP(kPiNone, true, static_cast<T*>(nullptr));
    else
      PDYN_LAUNCH_VJP(kPiNone, false, static_cast<T*>(nullptr));
  } else if (m->n_chains == 1) {
    PDYN_LAUNCH_VJP(kPiLanes, true, partials);
    hipLaunchKernelGGL(k_reduce_lanes<T>, dim3(m->n_links_max * 10), dim3(256), 0, s, b->n_states, partials,
                       inertia_bar);
  } else {
    PDYN_LAUNCH_VJP(kPiDirect, false, inertia_bar);
  }
#undef PDYN_LAUNCH_VJP
#undef PDYN_LAUNCH_VJP_SPLIT
  if (hipGetLastError() != hipSuccess) return PDYN_ELAUNCH;
  return PDYN_OK;
}

// Grid of the elementwise kernels: one thread per element, at most 8192 workgroups (grid-stride beyond).
unsigned elementwise_grid(int64_t n) {
  const int64_t g = (n + 255) / 256;
  return (unsigned)(g < 1 ? 1 : (g > 8192 ? 8192 : g));
}

template <class T>
int run_euler_step(int64_t n, double dt, T* q, T* qd, const T* qdd, void* stream) {
  if (n < 0 || !(dt == dt)) return PDYN_EINVAL;
  if (n == 0) return PDYN_OK;
  int st = check_ptrs<T>({q, qd, qdd});
  if (st) return st;
  hipLaunchKernelGGL(k_euler_step<T>, dim3(elementwise_grid(n)), dim3(256), 0, static_cast<hipStream_t>(stream), n,
                     (T)dt, q, qd, qdd);
  return hipGetLastError() == hipSuccess ? PDYN_OK : PDYN_ELAUNCH;
}

template <class T>
int run_euler_step_vjp(int64_t n, double dt, T* qb, T* qdb, const T* qbf, const T* qdbf, T* qddb, int64_t n_pi, T* pib,
                       const T* pibf, void* stream) {
  if (n < 0 || n_pi < 0 || !(dt == dt)) return PDYN_EINVAL;
  if ((qbf == nullptr) != (qdbf == nullptr)) return PDYN_EINVAL;
  if (pibf && !pib) return PDYN_EINVAL;
  int st = check_ptrs<T>({qb, qdb});
  if (n > 0 && st) return st;
  for (const void* p : {(const void*)qbf, (const void*)qdbf, (const void*)qddb, (const void*)pib, (const void*)pibf})
    if (p && !aligned(p, sizeof(T))) return PDYN_EALIGN;
  const int64_t m = n > n_pi || !pibf ? n : n_pi;
  if (m == 0) return PDYN_OK;
  hipLaunchKernelGGL(k_euler_step_vjp<T>, dim3(elementwise_grid(m)), dim3(256), 0, static_cast<hipStream_t>(stream),
                     n, (T)dt, qb, qdb, qbf, qdbf, qddb, n_pi, pib, pibf);
  return hipGetLastError() == hipSuccess ? PDYN_OK : PDYN_ELAUNCH;
}

// ---- the allocation-free entry point (pdyn_id_fd_noalloc) -----------------------------
//
// Its workspace is this file-scope array instead of caller memory: every device
// the library runs on holds one copy of it until the process ends. In host code
// the name is only a host-side handle of the symbol; its device address comes
// from hipGetSymbolAddress, taken once per device with that device current, and
// only that address is ever handed to kernels.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
static_assert(kNoAllocBytes == PDYN_NOALLOC_SCRATCH_BYTES, "static scratch size of the C ABI");
static __device__ __align__(256) unsigned char noalloc_scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mutex;
void* g_noalloc_ptr[kMaxDevices];

// Device address of noalloc_scratch on the current device.
int noalloc_scratch_ptr(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return PDYN_ELAUNCH;
  std::lock_guard<std::mutex> lock(g_noalloc_mutex);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(noalloc_scratch)) != hipSuccess || !p) return PDYN_ELAUNCH;
    g_noalloc_ptr[dev] = p;
  }
  *out = g_noalloc_ptr[dev];
  return PDYN_OK;
}

}  // namespace
}  // namespace pdyn

using namespace pdyn;

extern "C" {

int pdyn_read_status(void* ws, void* stream, uint32_t* bits) {
  if (!ws || !bits) return PDYN_EINVAL;
  if (!aligned(ws, kAlign)) return PDYN_EALIGN;
  hipStream_t s = static_cast<hipStream_t>(stream);
  uint32_t v = 0;
  if (hipMemcpyAsync(&v, ws, sizeof(v), hipMemcpyDeviceToHost, s) != hipSuccess) return PDYN_ELAUNCH;
  if (hipMemsetAsync(ws, 0, sizeof(v), s) != hipSuccess) return PDYN_ELAUNCH;
  if (hipStreamSynchronize(s) != hipSuccess) return PDYN_ELAUNCH;
  *bits = v;
  return PDYN_OK;
}

size_t pdyn_workspace_bytes(int op, const pdyn_model* model, const pdyn_batch* batch, int scalar_bytes) {
  if (scalar_bytes != 4 && scalar_bytes != 8) return 0;
  const bool scan_op = op == PDYN_OP_ARTICULATED_INERTIA || op == PDYN_OP_ABA_FD_SCAN;
  if (scan_op ? check_scan_batch(model, batch) : check_model_batch(model, batch)) return 0;
  if (op == PDYN_OP_RNEA_ID_JACOBIAN || op == PDYN_OP_ABA_FD_JACOBIAN) {
    JacLayout jl;
    if (model->n_chains != 1 ||
        jac_layout(op == PDYN_OP_RNEA_ID_JACOBIAN ? PDYN_OP_RNEA_ID_VJP : PDYN_OP_ABA_FD_VJP, model, batch,
                   (size_t)scalar_bytes, &jl))
      return 0;
    return jl.total;
  }
  if (op == PDYN_OP_RNEA_ID_HESSIAN) return model->n_chains == 1 ? hessian_ws_bytes(model, (size_t)scalar_bytes) : 0;
  if (op == PDYN_OP_ARTICULATED_INERTIA)
    return model->n_chains == 1 ? abi_scan_ws_bytes(model, (size_t)scalar_bytes) : 0;
  if (op == PDYN_OP_ABA_FD_SCAN)
    return model->n_chains == 1 ? fd_scan_ws_bytes(model, batch, (size_t)scalar_bytes, nullptr) : 0;
  if (op < PDYN_OP_RNEA_ID || op > PDYN_OP_MASS_MATRIX) return 0;
  const pdyn_batch bt = tuned_batch(op, model, batch, (size_t)scalar_bytes);  // the launch the call will take
  Layout L;
  if (layout_for(op, model, &bt, (size_t)scalar_bytes, &L)) return 0;
  return L.total;
}

size_t pdyn_model_prepared_bytes(const pdyn_model* model, int scalar_bytes) {
  if (scalar_bytes != 4 && scalar_bytes != 8) return 0;
  if (!model || model->n_chains < 1 || model->n_links_total < 1) return 0;
  return tables_bytes(model, (size_t)scalar_bytes, nullptr);
}

int pdyn_model_prepare(const pdyn_model* model, int scalar_bytes, void* prepared, size_t prepared_bytes,
                       void* stream) {
  if (scalar_bytes != 4 && scalar_bytes != 8) return PDYN_EINVAL;
  if (!model || model->n_chains < 1 || model->n_links_total < 1 || !prepared) return PDYN_EINVAL;
  if (!model->placement || !model->twist || !model->inertia) return PDYN_EINVAL;
  if (model->n_chains > 1 && !model->link_ptr) return PDYN_EINVAL;
  if (model->n_links_max < 1) return PDYN_EINVAL;
  if (model->n_links_max > kMaxLinks) return PDYN_EUNSUPPORTED;
  if (model->n_chains == 1 ? model->n_links_total != model->n_links_max : model->n_links_total > INT32_MAX)
    return model->n_chains == 1 ? PDYN_EINVAL : PDYN_EUNSUPPORTED;
  if (check_host_csr(model)) return PDYN_EINVAL;
  if (!aligned(prepared, kAlign) || (model->order && !aligned(model->order, sizeof(int32_t)))) return PDYN_EALIGN;
  size_t a = (size_t)scalar_bytes;
  if (!aligned(model->placement, a) || !aligned(model->twist, a) || !aligned(model->inertia, a)) return PDYN_EALIGN;
  if (prepared_bytes < tables_bytes(model, a, nullptr)) return PDYN_EWORKSPACE;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (scalar_bytes == 4) return launch_link_table<float>(model, static_cast<char*>(prepared), s);
  return launch_link_table<double>(model, static_cast<char*>(prepared), s);
}

int pdyn_max_links(void) { return kMaxLinks; }

int pdyn_launch_choice(int op, const pdyn_model* model, const pdyn_batch* batch, int scalar_bytes,
                       int32_t* block_threads, int32_t* max_blocks, int32_t* variant, int32_t* segments) {
  if (scalar_bytes != 4 && scalar_bytes != 8) return PDYN_EINVAL;
  if (op < PDYN_OP_RNEA_ID || op > PDYN_OP_MASS_MATRIX || !block_threads || !max_blocks || !variant || !segments)
    return PDYN_EINVAL;
  const int st = check_model_batch(model, batch);
  if (st) return st;
  const pdyn_batch b = tuned_batch(op, model, batch, (size_t)scalar_bytes);
  *block_threads = b.block_threads;
  *max_blocks = b.max_blocks;
  *variant = b.variant;
  *segments = b.variant == 4 ? team_lanes(model, &b, op) : b.segments;
  return PDYN_OK;
}

int pdyn_load_tuning(const char* json) {
  std::shared_ptr<const std::vector<TuneEntry>> tab;
  if (json && *json) {
    auto v = std::make_shared<std::vector<TuneEntry>>();
    const int st = parse_tuning(json, v.get());
    if (st) return st;
    tab = v;
  }
  std::lock_guard<std::mutex> lock(g_tune_mutex);
  g_tune = tab;
  return PDYN_OK;
}

const char* pdyn_strerror(int status) {
  switch (status) {
    case PDYN_OK: return "success";
    case PDYN_EINVAL: return "invalid argument";
    case PDYN_EALIGN: return "misaligned pointer";
    case PDYN_EWORKSPACE: return "workspace too small";
    case PDYN_ELAUNCH: return "kernel launch failed";
    case PDYN_EUNSUPPORTED: return "unsupported size";
    default: return "unknown status";
  }
}

int pdyn_rnea_id(const pdyn_model* m, const pdyn_batch* b, const float* q, const float* qd, const float* qdd,
                 float* tau, void* ws, size_t ws_bytes, void* stream) {
  return run_dynamics<float, kModeID>(PDYN_OP_RNEA_ID, m, b, q, qd, qdd, nullptr, tau, nullptr, ws, ws_bytes, stream);
}
int pdyn_rnea_id_f64(const pdyn_model* m, const pdyn_batch* b, const double* q, const double* qd, const double* qdd,
                     double* tau, void* ws, size_t ws_bytes, void* stream) {
  return run_dynamics<double, kModeID>(PDYN_OP_RNEA_ID, m, b, q, qd, qdd, nullptr, tau, nullptr, ws, ws_bytes, stream);
}
int pdyn_aba_fd(const pdyn_model* m, const pdyn_batch* b, const float* q, const float* qd, const float* tau,
                float* qdd, void* ws, size_t ws_bytes, void* stream) {
  return run_dynamics<float, kModeFD>(PDYN_OP_ABA_FD, m, b, q, qd, nullptr, tau, nullptr, qdd, ws, ws_bytes, stream);
}
int pdyn_aba_fd_f64(const pdyn_model* m, const pdyn_batch* b, const double* q, const double* qd, const double* tau,
                    double* qdd, void* ws, size_t ws_bytes, void* stream) {
  return run_dynamics<double, kModeFD>(PDYN_OP_ABA_FD, m, b, q, qd, nullptr, tau, nullptr, qdd, ws, ws_bytes, stream);
}
int pdyn_id_fd(const pdyn_model* m, const pdyn_batch* b, const float* q, const float* qd, const float* qdd_in,
               const float* tau_in, float* tau_out, float* qdd_out, void* ws, size_t ws_bytes, void* stream) {
  return run_dynamics<float, kModeIDFD>(PDYN_OP_ID_FD, m, b, q, qd, qdd_in, tau_in, tau_out, qdd_out, ws, ws_bytes, stream);
}
int pdyn_id_fd_f64(const pdyn_model* m, const pdyn_batch* b, const double* q, const double* qd, const double* qdd_in,
                   const double* tau_in, double* tau_out, double* qdd_out, void* ws, size_t ws_bytes, void* stream) {
  return run_dynamics<double, kModeIDFD>(PDYN_OP_ID_FD, m, b, q, qd, qdd_in, tau_in, tau_out, qdd_out, ws, ws_bytes, stream);
}

int pdyn_rnea_id_hessian(const pdyn_model* m, const pdyn_batch* b, const float* q, const float* qd,
                         const float* qdd, float* H_qq, float* H_qqd, float* H_qdqd, float* H_qqdd, void* ws,
                         size_t ws_bytes, void* stream) {
  return run_id_hessian<float>(m, b, q, qd, qdd, H_qq, H_qqd, H_qdqd, H_qqdd, ws, ws_bytes, stream);
}
int pdyn_rnea_id_hessian_f64(const pdyn_model* m, const pdyn_batch* b, const double* q, const double* qd,
                             const double* qdd, double* H_qq, double* H_qqd, double* H_qdqd, double* H_qqdd,
                             void* ws, size_t ws_bytes, void* stream) {
  return run_id_hessian<double>(m, b, q, qd, qdd, H_qq, H_qqd, H_qdqd, H_qqdd, ws, ws_bytes, stream);
}

int pdyn_articulated_inertia(const pdyn_model* m, const pdyn_batch* b, const float* q, float* Jhat, void* ws,
                             size_t ws_bytes, void* stream) {
  return run_abi_scan<float>(m, b, q, Jhat, ws, ws_bytes, stream);
}
int pdyn_articulated_inertia_f64(const pdyn_model* m, const pdyn_batch* b, const double* q, double* Jhat, void* ws,
                                 size_t ws_bytes, void* stream) {
  return run_abi_scan<double>(m, b, q, Jhat, ws, ws_bytes, stream);
}
int pdyn_aba_fd_scan(const pdyn_model* m, const pdyn_batch* b, const float* q, const float* qd, const float* tau,
                     float* qdd, void* ws, size_t ws_bytes, void* stream) {
  return run_fd_scan<float>(m, b, q, qd, tau, qdd, ws, ws_bytes, stream);
}
int pdyn_aba_fd_scan_f64(const pdyn_model* m, const pdyn_batch* b, const double* q, const double* qd,
                         const double* tau, double* qdd, void* ws, size_t ws_bytes, void* stream) {
  return run_fd_scan<double>(m, b, q, qd, tau, qdd, ws, ws_bytes, stream);
}
int pdyn_rnea_id_jacobian(const pdyn_model* m, const pdyn_batch* b, const float* q, const float* qd,
                          const float* qdd, float* J_q, float* J_qd, float* J_qdd, void* ws, size_t ws_bytes,
                          void* stream) {
  return run_jacobian<float, kVjpID>(m, b, q, qd, qdd, J_q, J_qd, J_qdd, ws, ws_bytes, stream);
}
int pdyn_rnea_id_jacobian_f64(const pdyn_model* m, const pdyn_batch* b, const double* q, const double* qd,
                              const double* qdd, double* J_q, double* J_qd, double* J_qdd, void* ws, size_t ws_bytes,
                              void* stream) {
  return run_jacobian<double, kVjpID>(m, b, q, qd, qdd, J_q, J_qd, J_qdd, ws, ws_bytes, stream);
}
int pdyn_aba_fd_jacobian(const pdyn_model* m, const pdyn_batch* b, const float* q, const float* qd,
                         const float* qdd, float* J_q, float* J_qd, float* J_tau, void* ws, size_t ws_bytes,
                         void* stream) {
  return run_jacobian<float, kVjpFD>(m, b, q, qd, qdd, J_q, J_qd, J_tau, ws, ws_bytes, stream);
}
int pdyn_aba_fd_jacobian_f64(const pdyn_model* m, const pdyn_batch* b, const double* q, const double* qd,
                             const double* qdd, double* J_q, double* J_qd, double* J_tau, void* ws, size_t ws_bytes,
                             void* stream) {
  return run_jacobian<double, kVjpFD>(m, b, q, qd, qdd, J_q, J_qd, J_tau, ws, ws_bytes, stream);
}

int pdyn_id_fd_noalloc(const pdyn_model* m, const pdyn_batch* b, const float* q, const float* qd,
                       const float* qdd_in, const float* tau_in, float* tau_out, float* qdd_out, uint32_t* status_out,
                       void* stream) {
  // every check that needs no device comes first, so a rejected call queues nothing
  const size_t need = pdyn_workspace_bytes(PDYN_OP_ID_FD, m, b, 4);
  if (need == 0) {
    const int st = check_model_batch(m, b);
    return st ? st : PDYN_EINVAL;
  }
  if (need > kNoAllocBytes) return PDYN_EWORKSPACE;
  if (status_out && !aligned(status_out, sizeof(uint32_t))) return PDYN_EALIGN;
  if (b->n_states == 0) return PDYN_OK;
  void* ws = nullptr;
  const int st = noalloc_scratch_ptr(&ws);
  if (st) return st;
  return run_dynamics<float, kModeIDFD>(PDYN_OP_ID_FD, m, b, q, qd, qdd_in, tau_in, tau_out, qdd_out, ws,
                                        kNoAllocBytes, stream, true, status_out);
}

int pdyn_mass_matrix(const pdyn_model* m, const pdyn_batch* b, const float* q, float* M, void* ws, size_t ws_bytes,
                     void* stream) {
  return run_jsiia<float, false>(m, b, q, nullptr, nullptr, M, ws, ws_bytes, stream);
}
int pdyn_mass_matrix_f64(const pdyn_model* m, const pdyn_batch* b, const double* q, double* M, void* ws,
                         size_t ws_bytes, void* stream) {
  return run_jsiia<double, false>(m, b, q, nullptr, nullptr, M, ws, ws_bytes, stream);
}
int pdyn_jsiia_fd(const pdyn_model* m, const pdyn_batch* b, const float* q, const float* qd, const float* tau,
                  float* qdd, void* ws, size_t ws_bytes, void* stream) {
  return run_jsiia<float, true>(m, b, q, qd, tau, qdd, ws, ws_bytes, stream);
}
int pdyn_jsiia_fd_f64(const pdyn_model* m, const pdyn_batch* b, const double* q, const double* qd,
                      const double* tau, double* qdd, void* ws, size_t ws_bytes, void* stream) {
  return run_jsiia<double, true>(m, b, q, qd, tau, qdd, ws, ws_bytes, stream);
}

int pdyn_rnea_id_vjp(const pdyn_model* m, const pdyn_batch* b, const float* q, const float* qd, const float* qdd,
                     const float* tau_bar, float* q_bar, float* qd_bar, float* qdd_bar, float* inertia_bar, void* ws,
                     size_t ws_bytes, void* stream) {
  return run_vjp<float, kVjpID>(m, b, q, qd, qdd, tau_bar, q_bar, qd_bar, qdd_bar, inertia_bar, ws, ws_bytes, stream);
}
int pdyn_rnea_id_vjp_f64(const pdyn_model* m, const pdyn_batch* b, const double* q, const double* qd,
                         const double* qdd, const double* tau_bar, double* q_bar, double* qd_bar, double* qdd_bar,
                         double* inertia_bar, void* ws, size_t ws_bytes, void* stream) {
  return run_vjp<double, kVjpID>(m, b, q, qd, qdd, tau_bar, q_bar, qd_bar, qdd_bar, inertia_bar, ws, ws_bytes, stream);
}
int pdyn_aba_fd_vjp(const pdyn_model* m, const pdyn_batch* b, const float* q, const float* qd, const float* qdd,
                    const float* qdd_bar, float* q_bar, float* qd_bar, float* tau_bar, float* inertia_bar, void* ws,
                    size_t ws_bytes, void* stream) {
  return run_vjp<float, kVjpFD>(m, b, q, qd, qdd, qdd_bar, q_bar, qd_bar, tau_bar, inertia_bar, ws, ws_bytes, stream);
}
int pdyn_aba_fd_vjp_f64(const pdyn_model* m, const pdyn_batch* b, const double* q, const double* qd,
                        const double* qdd, const double* qdd_bar, double* q_bar, double* qd_bar, double* tau_bar,
                        double* inertia_bar, void* ws, size_t ws_bytes, void* stream) {
  return run_vjp<double, kVjpFD>(m, b, q, qd, qdd, qdd_bar, q_bar, qd_bar, tau_bar, inertia_bar, ws, ws_bytes, stream);
}

size_t pdyn_rollout_workspace_bytes(int with_grad, const pdyn_model* model, const pdyn_batch* batch, int ckpt_every,
                                    int scalar_bytes) {
  if (scalar_bytes != 4 && scalar_bytes != 8) return 0;
  if (check_model_batch(model, batch) || ckpt_every < 1) return 0;
  size_t so, ro, ao;
  return rollout_layout(with_grad ? 1 : 0, model, batch, ckpt_every, (size_t)scalar_bytes, &so, &ro, &ao);
}

int pdyn_rollout(const pdyn_model* m, const pdyn_batch* b, int steps, double dt, int ckpt_every, const float* tau_seq,
                 float* q, float* qd, float* ckpt_q, float* ckpt_qd, void* ws, size_t ws_bytes, void* stream) {
  return run_rollout<float>(m, b, steps, dt, ckpt_every, tau_seq, q, qd, ckpt_q, ckpt_qd, ws, ws_bytes, stream);
}
int pdyn_rollout_f64(const pdyn_model* m, const pdyn_batch* b, int steps, double dt, int ckpt_every,
                     const double* tau_seq, double* q, double* qd, double* ckpt_q, double* ckpt_qd, void* ws,
                     size_t ws_bytes, void* stream) {
  return run_rollout<double>(m, b, steps, dt, ckpt_every, tau_seq, q, qd, ckpt_q, ckpt_qd, ws, ws_bytes, stream);
}
int pdyn_rollout_vjp(const pdyn_model* m, const pdyn_batch* b, int steps, double dt, int ckpt_every,
                     const float* tau_seq, const float* ckpt_q, const float* ckpt_qd, const float* qT_bar,
                     const float* qdT_bar, float* q0_bar, float* qd0_bar, float* tau_bar_seq, float* inertia_bar,
                     void* ws, size_t ws_bytes, void* stream) {
  return run_rollout_vjp<float>(m, b, steps, dt, ckpt_every, tau_seq, ckpt_q, ckpt_qd, qT_bar, qdT_bar, q0_bar,
                                qd0_bar, tau_bar_seq, inertia_bar, ws, ws_bytes, stream);
}
int pdyn_rollout_vjp_f64(const pdyn_model* m, const pdyn_batch* b, int steps, double dt, int ckpt_every,
                         const double* tau_seq, const double* ckpt_q, const double* ckpt_qd, const double* qT_bar,
                         const double* qdT_bar, double* q0_bar, double* qd0_bar, double* tau_bar_seq,
                         double* inertia_bar, void* ws, size_t ws_bytes, void* stream) {
  return run_rollout_vjp<double>(m, b, steps, dt, ckpt_every, tau_seq, ckpt_q, ckpt_qd, qT_bar, qdT_bar, q0_bar,
                                 qd0_bar, tau_bar_seq, inertia_bar, ws, ws_bytes, stream);
}

int pdyn_euler_step(int64_t n, double dt, float* q, float* qd, const float* qdd, void* stream) {
  return run_euler_step<float>(n, dt, q, qd, qdd, stream);
}
int pdyn_euler_step_f64(int64_t n, double dt, double* q, double* qd, const double* qdd, void* stream) {
  return run_euler_step<double>(n, dt, q, qd, qdd, stream);
}
int pdyn_euler_step_vjp(int64_t n, double dt, float* q_bar, float* qd_bar, const float* q_bar_fd,
                        const float* qd_bar_fd, float* qdd_bar, int64_t n_pi, float* pi_bar, const float* pi_bar_fd,
                        void* stream) {
  return run_euler_step_vjp<float>(n, dt, q_bar, qd_bar, q_bar_fd, qd_bar_fd, qdd_bar, n_pi, pi_bar, pi_bar_fd,
                                   stream);
}
int pdyn_euler_step_vjp_f64(int64_t n, double dt, double* q_bar, double* qd_bar, const double* q_bar_fd,
                            const double* qd_bar_fd, double* qdd_bar, int64_t n_pi, double* pi_bar,
                            const double* pi_bar_fd, void* stream) {
  return run_euler_step_vjp<double>(n, dt, q_bar, qd_bar, q_bar_fd, qd_bar_fd, qdd_bar, n_pi, pi_bar, pi_bar_fd,
                                    stream);
}

}  // extern "C"
