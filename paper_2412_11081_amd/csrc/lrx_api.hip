// Host side of the C-ABI declared in include/lrx.h.
//
// lrx_set_tensors builds, once per structure, the static work structure on
// the host (pairs of image blocks, H slots, triple offsets, work units) from
// the block keys, uploads it, and sizes every device buffer for the case
// where nothing is screened.  lrx_evaluate then runs only kernels: the
// screening decisions, folded blocks and slot needs are masks recomputed on
// the device every call, so a call never synchronises with the host before
// its results are copied back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <cstring>
#include <exception>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/lrx.h"
#include "lrx_internal.h"

using lrx::Dev;

// The fixed device scratch of lrx_evaluate_noalloc: one array per GPU, held
// from the module's load until the process ends.  Its name is only a
// host-side handle; host code uses the per-device address that
// hipGetSymbolAddress returns (scratch_on), never the name itself.
static __device__ __align__(256) unsigned char scratch[LRX_SCRATCH_BYTES];

namespace {

struct Fail {
  int code;
  std::string msg;
};

#define HIPCHK(x)                                                                         \
  do {                                                                                    \
    hipError_t e_ = (x);                                                                  \
    if (e_ != hipSuccess)                                                                 \
      throw Fail{e_ == hipErrorOutOfMemory ? LRX_ENOMEM : LRX_EHIP,                       \
                 std::string(#x) + ": " + hipGetErrorString(e_)};                         \
  } while (0)

inline void require(bool c, const std::string& msg) {
  if (!c) throw Fail{LRX_EINVAL, msg};
}

struct Key {
  int f, s, r0, r1, r2;
  bool operator<(const Key& o) const {
    return std::tie(f, s, r0, r1, r2) < std::tie(o.f, o.s, o.r0, o.r1, o.r2);
  }
  bool operator==(const Key& o) const { return f == o.f && s == o.s && r0 == o.r0 && r1 == o.r1 && r2 == o.r2; }
};

// Blocks of one tensor grouped into atom pairs (sorted by first, second, R).
struct Pairs {
  std::vector<int64_t> order;     // sorted position -> caller block index
  std::vector<int> pA, pB, b0, b1, row;
};

Pairs group_pairs(int N, int64_t n, const int32_t* first, const int32_t* second, const int32_t* R) {
  Pairs P;
  P.order.resize(n);
  std::iota(P.order.begin(), P.order.end(), 0);
  auto key = [&](int64_t b) { return Key{first[b], second[b], R[3 * b], R[3 * b + 1], R[3 * b + 2]}; };
  // the key packed into 64 bits with the same order (atoms below 2^20, image
  // indices in [-128, 127]), sorted with the block index; else the general sort
  bool packable = N <= (1 << 20);
  for (int64_t b = 0; b < n && packable; ++b)
    for (int x = 0; x < 3; ++x) packable = packable && R[3 * b + x] >= -128 && R[3 * b + x] <= 127;
  if (packable) {
    std::vector<std::pair<uint64_t, int64_t>> kv(n);
    for (int64_t b = 0; b < n; ++b)
      kv[b] = {(uint64_t)first[b] << 44 | (uint64_t)second[b] << 24 | (uint64_t)(R[3 * b] + 128) << 16 |
                   (uint64_t)(R[3 * b + 1] + 128) << 8 | (uint64_t)(R[3 * b + 2] + 128),
               b};
    std::sort(kv.begin(), kv.end());
    for (int64_t k = 0; k < n; ++k) P.order[k] = kv[k].second;
  } else {
    std::sort(P.order.begin(), P.order.end(), [&](int64_t a, int64_t b) { return key(a) < key(b); });
  }
  for (int64_t k = 1; k < n; ++k)
    require(!(key(P.order[k - 1]) == key(P.order[k])), "duplicate block key");
  P.row.assign(N + 1, 0);
  for (int64_t k = 0; k < n; ++k) {
    const int64_t b = P.order[k];
    if (k == 0 || first[b] != first[P.order[k - 1]] || second[b] != second[P.order[k - 1]]) {
      P.pA.push_back(first[b]);
      P.pB.push_back(second[b]);
      P.b0.push_back((int)k);
      P.b1.push_back((int)k + 1);
      P.row[first[b] + 1]++;
    } else {
      P.b1.back() = (int)k + 1;
    }
  }
  for (int i = 0; i < N; ++i) P.row[i + 1] += P.row[i];
  return P;
}

std::atomic<uint64_t> g_gen{1};

// Pinned host buffers for results, by power-of-two size class (4 KiB and up),
// kept for reuse: contexts that come and go (a serving stream) would otherwise
// pin and unpin host memory, and unpinning waits for the whole device.
struct PinnedPool {
  std::mutex mu;
  std::vector<std::vector<void*>> free_by_class = std::vector<std::vector<void*>>(40);
  static int size_class(size_t bytes) {
    int k = 12;
    while (((size_t)1 << k) < bytes) ++k;
    return k;
  }
  void* get(size_t bytes) {
    const int k = size_class(bytes);
    {
      std::lock_guard<std::mutex> lk(mu);
      if (!free_by_class[k].empty()) {
        void* p = free_by_class[k].back();
        free_by_class[k].pop_back();
        return p;
      }
    }
    void* p = nullptr;
    HIPCHK(hipHostMalloc(&p, (size_t)1 << k, hipHostMallocDefault));
    return p;
  }
  void put(void* p, size_t bytes) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(mu);
    free_by_class[size_class(bytes)].push_back(p);
  }
};
PinnedPool g_pinned;

// Non-blocking streams kept per device for reuse: contexts take theirs from
// here and give them back, synchronised, when destroyed, so contexts that come
// and go neither create nor destroy streams once the pool is warm, and memory
// a context frees stream-ordered is always ordered on a stream that lives on.
struct StreamPool {
  std::mutex mu;
  std::vector<std::pair<int, hipStream_t>> idle;
  hipStream_t get(int device) {
    {
      std::lock_guard<std::mutex> lk(mu);
      for (size_t k = idle.size(); k-- > 0;)
        if (idle[k].first == device) {
          hipStream_t s = idle[k].second;
          idle.erase(idle.begin() + k);
          return s;
        }
    }
    hipStream_t s = nullptr;
    HIPCHK(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    return s;
  }
  void put(int device, hipStream_t s) {
    if (!s) return;
    (void)hipStreamSynchronize(s);
    std::lock_guard<std::mutex> lk(mu);
    idle.emplace_back(device, s);
  }
};
StreamPool g_streams;

// CSR of blocks by atom (first or second), in caller order.
void by_atom(int N, int64_t n, const int32_t* atom, std::vector<int>& row, std::vector<int64_t>& list) {
  row.assign(N + 1, 0);
  for (int64_t b = 0; b < n; ++b) row[atom[b] + 1]++;
  for (int i = 0; i < N; ++i) row[i + 1] += row[i];
  list.resize(n);
  std::vector<int> fill(row.begin(), row.end() - 1);
  for (int64_t b = 0; b < n; ++b) list[fill[atom[b]]++] = b;
}

std::mutex g_scratch_mu;
std::map<int, unsigned char*> g_scratch_addr;   // device -> address of its scratch

// Address of this device's scratch, looked up once per device with that
// device current (called from lrx_create).
unsigned char* scratch_on(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) return it->second;
  void* p = nullptr;
  HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  if (!p) throw Fail{LRX_EHIP, "hipGetSymbolAddress(scratch) returned NULL"};
  g_scratch_addr[device] = (unsigned char*)p;
  return (unsigned char*)p;
}

__global__ void k_zero_u64(unsigned long long* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0ull;
}

}  // namespace

struct lrx_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;

  // structure
  int N = 0;
  std::vector<double> tau, lat;
  std::vector<int> nao, nabf;
  std::vector<int64_t> ao;
  double omega = 0;
  bool have_structure = false, have_tensors = false;

  // host copies of keys and static work structure
  int64_t nC = 0, nV = 0;
  std::vector<int32_t> Cf, Cs, CR, Vf, Vs, VR;
  Pairs cp, vp;
  std::vector<int> slotB, slotX, unitCp, unitK0, unitK1, unitKc, unitV0, unitV1, unitS, nkc, nsplit;
  std::vector<uint8_t> unitYonly;
  std::vector<uint8_t> vpZown;   // per V pair: 1 if this pair forms Z (of a pair and its mirror, exactly one)
  std::vector<int64_t> tBase;
  int max_mm = 1, max_depth = 4;
  // sizes of the FP32 buffers of the reduced-precision forms
  int64_t n_cf = 0, n_vf = 0, n_h = 0, n_z = 0, n_y = 0;
  bool have_f32 = false, have_f64 = false;
  // the Hamiltonian's buffers (allocated by its first call)
  bool have_hx = false;
  lrx::HxBufs hx{};
  double* hx_host_E = nullptr;            // pinned
  std::array<float, 5> hx_ms{};
  bool hx_timed = false;
  bool hx_done = false;

  // device memory
  std::vector<void*> allocs;
  double dev_bytes = 0;
  Dev dev{};
  uint64_t gen = 0;                       // changes whenever dev changes (batch plans key on it)
  std::vector<int> unitOrderHost;         // units sorted by alpha-tile group
  std::array<int, lrx::kMaxAlphaTiles + 2> mtStartHost{};
  lrx::TripleLaunch tl{};                 // this structure alone
  // autotuner result of the last batch plan built with this context first
  std::array<int, lrx::kMaxAlphaTiles + 1> tune_mode{};
  std::array<float, 2 * (lrx::kMaxAlphaTiles + 1)> tune_ms{};
  unsigned char* scratch = nullptr;   // this device's fixed scratch (lrx_evaluate_noalloc)
  double* h_out = nullptr;   // pinned, from g_pinned
  size_t h_out_bytes = 0;
  std::array<hipEvent_t, LRX_NSTAGES + 1> ev{};
  std::array<hipStream_t, lrx::kSideStreams> side{};
  std::array<hipEvent_t, lrx::kSideStreams + 1> fork{};
  bool events = false;
  std::array<float, LRX_NSTAGES> stage_ms{};
  std::array<hipEvent_t, 2 * (lrx::kMaxAlphaTiles + 1)> gev{};   // around each triple group's launch
  std::array<float, lrx::kMaxAlphaTiles + 1> group_ms{};
  bool timed = false;
  bool evaluated = false;
  bool per_tensor = false;   // screening mode of the last evaluation
  // k-point sampling (lrx_set_kpoint_tensors): the context then describes the
  // Born-von Karman supercell (N = N0 * cells atoms, atom (t, i) at t * N0 + i,
  // the home cell first) and keeps the unit cell here
  bool bvk = false;
  int nk[3] = {1, 1, 1};
  int N0 = 0;
  std::vector<double> tau0, lat0;
  std::vector<int> nao0, nabf0;
  std::vector<int64_t> ao0;
  const double* DscIm = nullptr;   // imaginary part of D(R) on the device (nullptr: a real D)
  double* keep2 = nullptr;   // gC, gV and out of the first real pass
  // evaluations queued by lrx_submit: results land in their own pinned buffer
  struct Ticket {
    hipEvent_t done = nullptr;
    double* h = nullptr;
    size_t bytes = 0;
    int N = 0;
  };
  std::map<int64_t, Ticket> tickets;
  int64_t next_ticket = 1;
  void release(Ticket& t) {
    if (t.done) (void)hipEventDestroy(t.done);
    g_pinned.put(t.h, t.bytes);
    t = Ticket{};
  }

  template <class T>
  T* dalloc(int64_t count) {
    void* p = nullptr;
    const size_t bytes = std::max<size_t>(1, (size_t)count * sizeof(T));
    // from the library's device memory cache: contexts that come and go (a
    // serving stream) reuse its memory instead of mapping fresh memory
    p = lrx::dev_alloc(device, bytes);
    if (!p) throw Fail{LRX_ENOMEM, "device memory exhausted (" + std::to_string(bytes) + " bytes requested)"};
    allocs.push_back(p);
    dev_bytes += (double)bytes;
    return (T*)p;
  }
  template <class T>
  T* upload(const std::vector<T>& v) {
    T* p = dalloc<T>((int64_t)v.size());
    if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, stream));
    return p;
  }
  void free_tensors() {
    // back to the cache once the work queued on this stream is done (every
    // call that uses the buffers on another stream has synchronised that
    // stream before returning)
    (void)hipStreamSynchronize(stream);
    for (void* p : allocs) lrx::dev_free(device, p);
    allocs.clear();
    dev_bytes = 0;
    have_tensors = false;
    have_f32 = have_f64 = false;
    have_hx = false;
    hx_done = false;
    evaluated = false;
    DscIm = nullptr;
    keep2 = nullptr;
  }
};

namespace {

void drop_plans_of(const lrx_ctx* c);   // batch plans that use c (defined with the batch code)

template <class F>
int guarded(lrx_ctx* ctx, F&& f) {
  if (!ctx) return LRX_EINVAL;
  try {
    HIPCHK(hipSetDevice(ctx->device));
    f();
    ctx->err.clear();
    return LRX_OK;
  } catch (const Fail& e) {
    ctx->err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    ctx->err = "host allocation failed";
    return LRX_ENOMEM;
  } catch (const std::exception& e) {
    ctx->err = e.what();
    return LRX_EINVAL;
  }
}

void check_blocks(const lrx_ctx* c, const lrx_blocks* B, bool isC, const char* name) {
  require(B != nullptr, std::string(name) + ": NULL");
  require(B->nblk >= 0 && B->nval >= 0, std::string(name) + ": negative size");
  if (B->nblk == 0) return;
  require(B->first && B->second && B->R && B->off && B->val && B->dval, std::string(name) + ": NULL array");
  for (int64_t b = 0; b < B->nblk; ++b) {
    const int f = B->first[b], s = B->second[b];
    require(f >= 0 && f < c->N && s >= 0 && s < c->N, std::string(name) + ": atom index out of range");
    const int64_t sz = isC ? (int64_t)c->nabf[f] * c->nao[f] * c->nao[s] : (int64_t)c->nabf[f] * c->nabf[s];
    require(B->off[b] >= 0 && B->off[b] + sz <= B->nval, std::string(name) + ": block exceeds nval");
  }
}

// The supercell of k-point sampling as the host list build sees it: atom
// (t, i) at index t * N0 + i, cell t = t0 + nk0 (t1 + nk1 t2).
struct KMap {
  int N0 = 0;
  int nk[3] = {1, 1, 1};
  const int32_t* VR0 = nullptr;   // the caller's lattice indices of the V blocks (mirror check)
  const double* Dim = nullptr;    // imaginary part of the supercell D on the device, or nullptr
  int home(int a) const { return a % N0; }
  int cell(int a) const { return a / N0; }
  // the cell offset u - t of cells u and t (modulo nk)
  int diff(int u, int t) const {
    const int u0 = u % nk[0], u1 = (u / nk[0]) % nk[1], u2 = u / (nk[0] * nk[1]);
    const int t0 = t % nk[0], t1 = (t / nk[0]) % nk[1], t2 = t / (nk[0] * nk[1]);
    return (u0 - t0 + nk[0]) % nk[0] + nk[0] * ((u1 - t1 + nk[1]) % nk[1] + nk[1] * ((u2 - t2 + nk[2]) % nk[2]));
  }
  // atom a moved back by the cell of atom b (cell(a) - cell(b) modulo nk)
  int back(int a, int b) const { return diff(cell(a), cell(b)) * N0 + home(a); }
};

// The static work structure of one set of tensors (keys checked by the
// caller): pairs, H slots, work units, offsets; device buffers; value checks.
// km == nullptr: the Gamma point.  Otherwise the context describes the BvK
// supercell, every block's first atom lies in the home cell, and D is the
// dense supercell matrix (real part; km->Dim the imaginary part).
void build_tensors(lrx_ctx* c, const lrx_blocks* C, const lrx_blocks* V, const double* D, bool d_on_device,
                   bool on_device, const KMap* km) {
  const int N = c->N;
  const int64_t ntot = c->ao[N];
  // rows of D are addressed with 24-bit byte strides inside the kernels
  require(ntot * (int64_t)sizeof(double) < (int64_t)1 << 24, "D: more than 2097151 NAOs in the cell");
  const int Nh = km ? km->N0 : N;   // atoms of the home cell (the atoms of every C and V block's first index)
  // D row/column index of AO x of atom X in the H-build tables: at the Gamma
  // point the index in the dense D; with k-point sampling the atom's cell
  // (bits 21 and up) and the AO index within the unit cell (d_block reads
  // the block of the cells' offset)
  auto dindex = [&](int X, int x) -> int {
    return km ? (km->cell(X) << 21) | (int)(c->ao0[km->home(X)] + x) : (int)(c->ao[X] + x);
  };
  c->nC = C->nblk;
  c->nV = V->nblk;
  c->Cf.assign(C->first, C->first + c->nC);
  c->Cs.assign(C->second, C->second + c->nC);
  c->CR.assign(C->R, C->R + 3 * c->nC);
  c->Vf.assign(V->first, V->first + c->nV);
  c->Vs.assign(V->second, V->second + c->nV);
  c->VR.assign(V->R, V->R + 3 * c->nV);

  // ---- pairs ---------------------------------------------------------
  c->cp = group_pairs(N, c->nC, C->first, C->second, C->R);
  c->vp = group_pairs(N, c->nV, V->first, V->second, V->R);
  const Pairs& cp = c->cp;
  const Pairs& vp = c->vp;
  const int nCp = (int)cp.pA.size(), nVp = (int)vp.pA.size();
  {  // every atom has its on-site C block
    std::vector<char> on(N, 0);
    for (int64_t b = 0; b < c->nC; ++b)
      if (C->first[b] == C->second[b] && !C->R[3 * b] && !C->R[3 * b + 1] && !C->R[3 * b + 2]) on[C->first[b]] = 1;
    for (int i = 0; i < Nh; ++i) require(on[i], "C: atom " + std::to_string(i) + " has no on-site block (A,A,0)");
  }
  // mirror of every V block: (B, A, -R) for (A, B, R).  The blocks of a pair
  // are sorted by R, so the mirrors of pair (A,B)'s blocks are pair (B,A)'s
  // blocks in reverse order; every pairing is checked.  On a k-point
  // supercell the mirror is moved back into the home cell: pair (A, (t, B))
  // has the mirror (B, (-t, A)), whose lattice indices are again sorted in
  // reverse order (the caller's R is checked).
  const int32_t* VR0 = km ? km->VR0 : V->R;
  std::vector<int64_t> vmir(c->nV);
  std::vector<int> vpmir(nVp);
  for (int p = 0; p < nVp; ++p) {
    const int A = vp.pA[p], B = vp.pB[p];
    const int mf = km ? km->home(B) : B, ms = km ? km->back(A, B) : A;
    const auto beg = vp.pB.begin() + vp.row[mf], end = vp.pB.begin() + vp.row[mf + 1];
    const auto it = std::lower_bound(beg, end, ms);
    require(it != end && *it == ms, "V: block without its mirror (second, first, -R)");
    const int pm = (int)(it - vp.pB.begin());
    const int n = vp.b1[p] - vp.b0[p];
    require(vp.b1[pm] - vp.b0[pm] == n, "V: block without its mirror (second, first, -R)");
    vpmir[p] = pm;
    for (int j = 0; j < n; ++j) {
      const int64_t b = vp.order[vp.b0[p] + j], bm = vp.order[vp.b1[pm] - 1 - j];
      require(V->first[bm] == mf && V->second[bm] == ms && VR0[3 * bm] == -VR0[3 * b] &&
                  VR0[3 * bm + 1] == -VR0[3 * b + 1] && VR0[3 * bm + 2] == -VR0[3 * b + 2],
              "V: block without its mirror (second, first, -R)");
      vmir[b] = bm;
    }
  }
  // Z(B,A) = Z(A,B)^T: of a pair and its mirror the one with the lower index
  // forms Z and writes both pairs' energy terms and V gradients (at the Gamma
  // point: the pair with B >= A).  The V pairs of every atom are then put in
  // the order (forms Z, partner), so the pairs that form Z are one range and a
  // work unit forms Z for all of its V pairs or for none.  At the Gamma point
  // that order is the sorted order.
  {
    std::vector<uint8_t> zown(nVp);
    for (int p = 0; p < nVp; ++p) zown[p] = p <= vpmir[p];
    std::vector<int> perm(nVp);   // new position -> pair in sorted order
    bool moved = false;
    for (int A = 0; A < N; ++A) {
      int k = vp.row[A];
      for (int z = 0; z < 2; ++z)
        for (int p = vp.row[A]; p < vp.row[A + 1]; ++p)
          if (zown[p] == z) {
            moved = moved || p != k;
            perm[k++] = p;
          }
    }
    if (moved) {
      std::vector<int> inv(nVp), mir(nVp);
      for (int q = 0; q < nVp; ++q) inv[perm[q]] = q;
      Pairs w = vp;
      std::vector<uint8_t> z2(nVp);
      for (int q = 0; q < nVp; ++q) {
        const int o = perm[q];
        w.pA[q] = vp.pA[o];
        w.pB[q] = vp.pB[o];
        w.b0[q] = vp.b0[o];
        w.b1[q] = vp.b1[o];
        mir[q] = inv[vpmir[o]];
        z2[q] = zown[o];
      }
      c->vp = std::move(w);
      vpmir = std::move(mir);
      zown = std::move(z2);
    }
    c->vpZown = std::move(zown);
  }
  const std::vector<uint8_t>& zown = c->vpZown;
  // ---- per-pair sizes and offsets --------------------------------------
  std::vector<int64_t> cfOff(nCp + 1, 0), vfOff(nVp + 1, 0);
  for (int i = 0; i < nCp; ++i)
    cfOff[i + 1] = cfOff[i] + (int64_t)c->nabf[cp.pA[i]] * c->nao[cp.pA[i]] * c->nao[cp.pB[i]];
  int max_mm = 1;
  for (int i = 0; i < nVp; ++i) {
    const int mm = c->nabf[vp.pA[i]] * c->nabf[vp.pB[i]];
    vfOff[i + 1] = vfOff[i] + (int64_t)c->nabf[vp.pA[i]] * ((c->nabf[vp.pB[i]] + 15) & ~15);   // rows padded
    max_mm = std::max(max_mm, mm);
  }
  c->max_mm = max_mm;
  // ---- H slots: (B,F) and (B,A) for every candidate triple (A,F,B) -----
  // On a k-point supercell H(B,X) depends only on the cells' offset: the
  // slot of (B, X) is that of (B in the home cell, X moved back by B's
  // cell), so slots are formed for home-cell atoms B only and slotmap sends
  // every (B, X) to its home slot.
  std::vector<int> slotmap((size_t)N * N, -1);
  {
    auto home_pair = [&](int B, int X) -> size_t {
      return km ? (size_t)km->home(B) * N + km->back(X, B) : (size_t)B * N + X;
    };
    std::vector<char> needm((size_t)Nh * N, 0);
    for (int i = 0; i < nCp; ++i) {
      const int A = cp.pA[i], F = cp.pB[i];
      for (int p = vp.row[A]; p < vp.row[A + 1]; ++p) {
        const int B = vp.pB[p];
        needm[home_pair(B, F)] = 1;
        needm[home_pair(B, A)] = 1;
      }
    }
    c->slotB.clear();
    c->slotX.clear();
    std::vector<int> home_slot((size_t)Nh * N, -1);
    for (int B = 0; B < Nh; ++B)
      for (int X = 0; X < N; ++X)
        if (needm[(size_t)B * N + X]) {
          home_slot[(size_t)B * N + X] = (int)c->slotB.size();
          c->slotB.push_back(B);
          c->slotX.push_back(X);
        }
    for (int B = 0; B < N; ++B)
      for (int X = 0; X < N; ++X) slotmap[(size_t)B * N + X] = home_slot[home_pair(B, X)];
  }
  const int nSlot = (int)c->slotB.size();
  std::vector<int64_t> hOff(nSlot + 1, 0);
  for (int s = 0; s < nSlot; ++s) {
    const int B = c->slotB[s], X = c->slotX[s];
    hOff[s + 1] = hOff[s] + (int64_t)((c->nabf[B] + 15) / 16 * 16) * c->nao[B] * c->nao[X];
  }
  std::vector<int> slotRow(N + 1, 0), hbB, hbR0, hbC0, hColRow(N + 1, 0), hColSlot, hColX, hColD, hColAtom;
  for (int s = 0; s < nSlot; ++s) slotRow[c->slotB[s] + 1]++;
  for (int B = 0; B < N; ++B) slotRow[B + 1] += slotRow[B];
  c->max_depth = 4;
  for (int B = 0; B < N; ++B) {  // depth of every H build fits the kernel's table
    int k = 0;
    for (int i = cp.row[B]; i < cp.row[B + 1]; ++i) k += c->nao[cp.pB[i]];
    require(k + 3 <= lrx::kHMaxDepth,
            "atom " + std::to_string(B) + ": its C partners have more than 508 NAOs in total");
    c->max_depth = std::max(c->max_depth, (k + 3) & ~3);
  }
  {
    int64_t ncol = 0;
    for (int s = 0; s < nSlot; ++s) ncol += c->nao[c->slotX[s]];
    hColSlot.reserve(ncol);
    hColX.reserve(ncol);
    hColD.reserve(ncol);
    hColAtom.reserve(ncol);
  }
  for (int B = 0; B < N; ++B) {
    for (int s = slotRow[B]; s < slotRow[B + 1]; ++s)
      for (int x = 0; x < c->nao[c->slotX[s]]; ++x) {
        hColSlot.push_back(s);
        hColX.push_back(x);
        hColD.push_back(dindex(c->slotX[s], x));
        hColAtom.push_back(c->slotX[s]);
      }
    hColRow[B + 1] = (int)hColSlot.size();
    const int rows = c->nabf[B] * c->nao[B], cols = hColRow[B + 1] - hColRow[B];
    for (int r0 = 0; r0 < rows; r0 += lrx::kHRows)
      for (int c0 = 0; c0 < cols; c0 += lrx::kHItemCols) {
        hbB.push_back(B);
        hbR0.push_back(r0);
        hbC0.push_back(c0);
      }
  }
  // ---- work units and triple offsets -----------------------------------
  c->unitCp.clear(); c->unitK0.clear(); c->unitK1.clear(); c->unitKc.clear();
  c->unitV0.clear(); c->unitV1.clear(); c->unitS.clear();
  c->nkc.assign(nCp, 1);
  // B-split: the V partners of a C pair are divided into nsplit ranges (Y
  // partials summed later) so every alpha-tile group has enough units to
  // fill the device.
  c->nsplit.assign(nCp, 1);
  {
    std::vector<int64_t> per_mt(lrx::kMaxAlphaTiles + 2, 0);
    for (int i = 0; i < nCp; ++i) {
      const int K1 = c->nao[cp.pA[i]] * c->nao[cp.pB[i]];
      const int mt = (c->nabf[cp.pA[i]] + 15) / 16;
      const int cols = lrx::unit_cols(mt);
      per_mt[mt] += (K1 + cols - 1) / cols;
    }
    for (int i = 0; i < nCp; ++i) {
      const int mt = (c->nabf[cp.pA[i]] + 15) / 16;
      const int nv = vp.row[cp.pA[i] + 1] - vp.row[cp.pA[i]];
      const int64_t want = (3 * 256 + per_mt[mt] - 1) / std::max<int64_t>(1, per_mt[mt]);
      c->nsplit[i] = (int)std::max<int64_t>(1, std::min<int64_t>({want, (int64_t)nv, 16}));
    }
  }
  // The V partners of A fall in two ranges: the pairs whose mirror forms Z,
  // where only Y is formed (Z(A,B) is the transpose of the mirror's Z,
  // formed by the units of the mirror's atom; at the Gamma point B < A), and
  // the pairs that form Z, where Z and Y are both formed.  Each range is
  // divided into its share of the C pair's nsplit V ranges.
  c->unitYonly.clear();
  for (int i = 0; i < nCp; ++i) {
    const int K1 = c->nao[cp.pA[i]] * c->nao[cp.pB[i]];
    const int cols = lrx::unit_cols((c->nabf[cp.pA[i]] + 15) / 16);
    const int nk = (K1 + cols - 1) / cols;
    int chunk = (K1 + nk - 1) / nk;
    chunk = std::min(cols, (chunk + 15) / 16 * 16);
    int cnt = 0;
    const int A = cp.pA[i];
    const int r0 = vp.row[A], r1 = vp.row[A + 1], nv = r1 - r0, ns = c->nsplit[i];
    int mid = r0;
    while (mid < r1 && !zown[mid]) ++mid;
    const int ny = mid - r0, nz = r1 - mid;
    const int nsY = ny > 0 ? std::max(1, (int)(((int64_t)ns * ny + nv / 2) / std::max(1, nv))) : 0;
    const int nsZ = nz > 0 ? std::max(1, ns - nsY) : 0;
    for (int k0 = 0; k0 < K1; k0 += chunk, ++cnt)
      for (int sp = 0; sp < nsY + nsZ; ++sp) {
        const bool yo = sp < nsY;
        const int b0 = yo ? r0 : mid, len = yo ? ny : nz, m = yo ? nsY : nsZ, k = yo ? sp : sp - nsY;
        c->unitCp.push_back(i);
        c->unitK0.push_back(k0);
        c->unitK1.push_back(std::min(K1, k0 + chunk));
        c->unitKc.push_back(cnt);
        c->unitV0.push_back(b0 + (int)((int64_t)len * k / m));
        c->unitV1.push_back(b0 + (int)((int64_t)len * (k + 1) / m));
        c->unitS.push_back(sp);
        c->unitYonly.push_back(yo ? 1 : 0);
      }
    c->nkc[i] = cnt;
    c->nsplit[i] = nsY + nsZ;
  }
  for (int A = 0; A < N; ++A) {
    int z = 0;
    for (int i = cp.row[A]; i < cp.row[A + 1]; ++i) z += c->nkc[i];
    require(z <= 64, "atom " + std::to_string(A) + ": more than 64 C-pair column chunks");
  }
  c->tBase.assign(N + 1, 0);
  for (int A = 0; A < N; ++A)
    c->tBase[A + 1] = c->tBase[A] + (int64_t)(cp.row[A + 1] - cp.row[A]) * (vp.row[A + 1] - vp.row[A]);
  const int64_t ntri = c->tBase[N];
  std::vector<int64_t> zOff(ntri + 1, 0);
  for (int A = 0; A < N; ++A) {
    const int nvA = vp.row[A + 1] - vp.row[A];
    for (int i = cp.row[A]; i < cp.row[A + 1]; ++i)
      for (int p = vp.row[A]; p < vp.row[A + 1]; ++p) {
        const int64_t t = c->tBase[A] + (int64_t)(i - cp.row[A]) * nvA + (p - vp.row[A]);
        // Z partials only where Z(A,B) is formed
        zOff[t + 1] = zown[p] ? (int64_t)c->nkc[i] * c->nabf[A] * c->nabf[vp.pB[p]] : 0;
      }
  }
  for (int64_t t = 0; t < ntri; ++t) zOff[t + 1] += zOff[t];
  std::vector<int64_t> triHF(std::max<int64_t>(1, ntri)), triHA(std::max<int64_t>(1, ntri));
  for (int A = 0; A < N; ++A) {
    const int nvA = vp.row[A + 1] - vp.row[A];
    for (int i = cp.row[A]; i < cp.row[A + 1]; ++i)
      for (int p = vp.row[A]; p < vp.row[A + 1]; ++p) {
        const int64_t t = c->tBase[A] + (int64_t)(i - cp.row[A]) * nvA + (p - vp.row[A]);
        const int B = vp.pB[p];
        triHF[t] = hOff[slotmap[(size_t)B * N + cp.pB[i]]];
        triHA[t] = hOff[slotmap[(size_t)B * N + A]];
      }
  }
  // static depth tables of the H build: every g of every C pair (B, G)
  std::vector<int> hdRow(N + 1, 0), hdRowD, hdG, hdCp, hdStride;
  std::vector<int64_t> hdCf;
  for (int B = 0; B < N; ++B) {
    int k = 0;
    for (int i = cp.row[B]; i < cp.row[B + 1]; ++i)
      for (int gg = 0; gg < c->nao[cp.pB[i]]; ++gg, ++k) {
        hdRowD.push_back(dindex(cp.pB[i], gg));
        hdG.push_back(cp.pB[i]);
        hdCp.push_back((i << 6) | gg);
        hdCf.push_back(cfOff[i] + gg);
        hdStride.push_back(c->nao[cp.pB[i]]);
      }
    // padding to a multiple of 4 entries, at least 4 (atoms outside the
    // home cell of a k-point supercell have no C pairs)
    for (; (k & 3) || k == 0; ++k) {
      hdRowD.push_back(0);
      hdG.push_back(-1);
      hdCp.push_back(-1);
      hdCf.push_back(0);
      hdStride.push_back(0);
    }
    hdRow[B + 1] = (int)hdRowD.size();
  }
  // ---- per-atom block lists for the force reduction ---------------------
  std::vector<int> atCfRow, atCsRow, atVfRow, atVsRow;
  std::vector<int64_t> atCf, atCs, atVf, atVs;
  // (on a k-point supercell the second atom counts for its home-cell atom:
  // the forces per unit cell)
  std::vector<int32_t> homeCs, homeVs;
  const int32_t* Cs_at = C->second;
  const int32_t* Vs_at = V->second;
  if (km) {
    homeCs.resize(c->nC);
    homeVs.resize(c->nV);
    for (int64_t b = 0; b < c->nC; ++b) homeCs[b] = km->home(C->second[b]);
    for (int64_t b = 0; b < c->nV; ++b) homeVs[b] = km->home(V->second[b]);
    Cs_at = homeCs.data();
    Vs_at = homeVs.data();
  }
  by_atom(N, c->nC, C->first, atCfRow, atCf);
  by_atom(N, c->nC, Cs_at, atCsRow, atCs);
  by_atom(N, c->nV, V->first, atVfRow, atVf);
  by_atom(N, c->nV, Vs_at, atVsRow, atVs);
  std::vector<int> Csz(c->nC), Vsz(c->nV);
  for (int64_t b = 0; b < c->nC; ++b) Csz[b] = c->nabf[C->first[b]] * c->nao[C->first[b]] * c->nao[C->second[b]];
  for (int64_t b = 0; b < c->nV; ++b) Vsz[b] = c->nabf[V->first[b]] * c->nabf[V->second[b]];

  // ---- device buffers ----------------------------------------------------
  Dev& d = c->dev;
  d = Dev{};
  d.N = N;
  d.ntot = ntot;
  d.omega = c->omega;
  d.tau = c->upload(c->tau);
  d.lat = c->upload(c->lat);
  d.nao = c->upload(c->nao);
  d.nabf = c->upload(c->nabf);
  d.ao = c->upload(c->ao);
  d.nC = c->nC;
  d.nV = c->nV;
  d.Cfirst = c->upload(c->Cf);
  d.Csecond = c->upload(c->Cs);
  d.CR = c->upload(c->CR);
  d.Coff = c->upload(std::vector<int64_t>(C->off, C->off + c->nC));
  d.Csz = c->upload(Csz);
  d.Vfirst = c->upload(c->Vf);
  d.Vsecond = c->upload(c->Vs);
  d.VR = c->upload(c->VR);
  d.Voff = c->upload(std::vector<int64_t>(V->off, V->off + c->nV));
  d.Vsz = c->upload(Vsz);
  d.Vmir = c->upload(vmir);
  if (on_device) {
    d.Cval = C->val; d.Cdval = C->dval; d.Vval = V->val; d.Vdval = V->dval;
  } else {
    double* p;
    p = c->dalloc<double>(C->nval); HIPCHK(hipMemcpyAsync(p, C->val, C->nval * 8, hipMemcpyHostToDevice, c->stream)); d.Cval = p;
    p = c->dalloc<double>(3 * C->nval); HIPCHK(hipMemcpyAsync(p, C->dval, 3 * C->nval * 8, hipMemcpyHostToDevice, c->stream)); d.Cdval = p;
    p = c->dalloc<double>(V->nval); HIPCHK(hipMemcpyAsync(p, V->val, V->nval * 8, hipMemcpyHostToDevice, c->stream)); d.Vval = p;
    p = c->dalloc<double>(3 * V->nval); HIPCHK(hipMemcpyAsync(p, V->dval, 3 * V->nval * 8, hipMemcpyHostToDevice, c->stream)); d.Vdval = p;
  }
  if (d_on_device) {
    d.D = D;
  } else {
    double* p = c->dalloc<double>(ntot * ntot);
    HIPCHK(hipMemcpyAsync(p, D, ntot * ntot * 8, hipMemcpyHostToDevice, c->stream));
    d.D = p;
  }
  d.DnRe = d.D;
  d.DnIm = km ? km->Dim : nullptr;
  {
    std::vector<int> acell(N, 0), dsub(1, 0);
    std::vector<int64_t> aloc(c->ao.begin(), c->ao.begin() + N);
    d.ncell = 1;
    d.dld = ntot;
    d.dcellsz = 0;
    d.dsize = ntot * ntot;
    if (km) {
      const int nc = km->nk[0] * km->nk[1] * km->nk[2];
      const int64_t nt0 = c->ao0[km->N0];
      for (int a = 0; a < N; ++a) {
        acell[a] = km->cell(a);
        aloc[a] = c->ao0[km->home(a)];
      }
      dsub.assign((size_t)nc * nc, 0);
      for (int t = 0; t < nc; ++t)
        for (int u = 0; u < nc; ++u) dsub[(size_t)t * nc + u] = km->diff(u, t);
      d.ncell = nc;
      d.dld = nt0;
      d.dcellsz = nt0 * nt0;
      d.dsize = nc * nt0 * nt0;
    }
    d.acell = c->upload(acell);
    d.aloc = c->upload(aloc);
    d.dsub = c->upload(dsub);
  }
  d.nCp = nCp;
  d.nVp = nVp;
  std::vector<int64_t> cpBlk(cp.order), vpBlk(vp.order);
  d.cpA = c->upload(cp.pA); d.cpF = c->upload(cp.pB); d.cpB0 = c->upload(cp.b0); d.cpB1 = c->upload(cp.b1);
  d.cpBlk = c->upload(cpBlk); d.cpRow = c->upload(cp.row);
  d.vpA = c->upload(vp.pA); d.vpB = c->upload(vp.pB); d.vpB0 = c->upload(vp.b0); d.vpB1 = c->upload(vp.b1);
  d.vpBlk = c->upload(vpBlk); d.vpRow = c->upload(vp.row); d.vpMir = c->upload(vpmir);
  d.vpZ = c->upload(zown);
  d.cfOff = c->upload(cfOff); d.vfOff = c->upload(vfOff);
  d.Cf = c->dalloc<double>(cfOff[nCp]);
  d.Vf = c->dalloc<double>(vfOff[nVp]);
  d.nrmC = c->dalloc<double>(4 * c->nC);
  d.nrmV = c->dalloc<double>(4 * c->nV);
  d.dmax = c->dalloc<double>((int64_t)N * N);
  d.dss = c->dalloc<double>((int64_t)N * N);
  d.keepC = c->dalloc<uint8_t>(c->nC);
  d.keepV = c->dalloc<uint8_t>(c->nV);
  d.keepD = c->dalloc<uint8_t>((int64_t)N * N);
  d.cval = c->dalloc<double>(nCp);
  d.dnrm = c->dalloc<double>((int64_t)N * N);
  d.Svp = c->dalloc<double>(nVp);
  d.aliveC = c->dalloc<uint8_t>(nCp);
  d.aliveV = c->dalloc<uint8_t>(nVp);
  d.nSlot = nSlot;
  d.slotB = c->upload(c->slotB); d.slotX = c->upload(c->slotX); d.hOff = c->upload(hOff);
  d.hSlotMap = c->upload(slotmap);
  {
    // counting sort by X, stable: slots of one X keep their (B) order
    std::vector<int> at(N + 1, 0), byX(nSlot);
    for (int s = 0; s < nSlot; ++s) at[c->slotX[s] + 1]++;
    for (int x = 0; x < N; ++x) at[x + 1] += at[x];
    for (int s = 0; s < nSlot; ++s) byX[at[c->slotX[s]]++] = s;
    d.slotByX = c->upload(byX);
  }
  d.need = c->dalloc<uint8_t>(nSlot);
  d.H = nullptr;   // work buffers of a precision are allocated on its first evaluation
  c->n_cf = cfOff[nCp];
  c->n_vf = vfOff[nVp];
  c->n_h = hOff[nSlot];

  d.nUnit = (int)c->unitCp.size();
  std::vector<int> unitOrder(d.nUnit);
  {
    std::iota(unitOrder.begin(), unitOrder.end(), 0);
    auto mt = [&](int u) { return (c->nabf[cp.pA[c->unitCp[u]]] + 15) / 16; };
    std::stable_sort(unitOrder.begin(), unitOrder.end(), [&](int a, int b) { return mt(a) < mt(b); });
    for (int m = 0; m <= lrx::kMaxAlphaTiles + 1; ++m) d.mtStart[m] = 0;
    for (int u = 0; u < d.nUnit; ++u) d.mtStart[mt(u) + 1]++;
    for (int m = 0; m <= lrx::kMaxAlphaTiles; ++m) d.mtStart[m + 1] += d.mtStart[m];
  }
  d.unitOrder = c->upload(unitOrder);
  c->unitOrderHost = unitOrder;
  for (int m = 0; m <= lrx::kMaxAlphaTiles + 1; ++m) c->mtStartHost[m] = d.mtStart[m];
  {
    std::vector<int2> items(d.nUnit);
    for (int k = 0; k < d.nUnit; ++k) items[k] = make_int2(0, unitOrder[k]);
    int2* it = c->upload(items);
    c->tl = lrx::TripleLaunch{};
    for (int mt = 1; mt <= lrx::kMaxAlphaTiles; ++mt) {
      c->tl.items[mt] = it + d.mtStart[mt];
      c->tl.n[mt] = d.mtStart[mt + 1] - d.mtStart[mt];
    }
    c->tl.counters = c->dalloc<int>(8 * (lrx::kMaxAlphaTiles + 1));
  }
  d.slotRow = c->upload(slotRow);
  d.nHB = (int)hbB.size();
  d.hbB = c->upload(hbB);
  d.hbR0 = c->upload(hbR0);
  d.hbC0 = c->upload(hbC0);
  d.hColRow = c->upload(hColRow);
  d.hColSlot = c->upload(hColSlot);
  d.hColX = c->upload(hColX);
  d.hColD = c->upload(hColD);
  d.hColAtom = c->upload(hColAtom);
  d.unitCp = c->upload(c->unitCp); d.unitK0 = c->upload(c->unitK0); d.unitK1 = c->upload(c->unitK1);
  d.unitKc = c->upload(c->unitKc); d.nkc = c->upload(c->nkc);
  d.unitV0 = c->upload(c->unitV0); d.unitV1 = c->upload(c->unitV1); d.unitS = c->upload(c->unitS);
  d.unitYonly = c->upload(c->unitYonly);
  d.unitRole = c->dalloc<uint8_t>((int64_t)c->unitYonly.size());
  d.nsplit = c->upload(c->nsplit);
  d.tBase = c->upload(c->tBase); d.zOff = c->upload(zOff);
  d.triHF = c->upload(triHF); d.triHA = c->upload(triHA);
  d.hdRow = c->upload(hdRow); d.hdRowD = c->upload(hdRowD); d.hdG = c->upload(hdG); d.hdCp = c->upload(hdCp);
  d.hdCf = c->upload(hdCf); d.hdStride = c->upload(hdStride);
  d.hcK = c->dalloc<int>(N);
  d.hcNcol = c->dalloc<int>(N);
  d.hcRowD = c->dalloc<int>((int64_t)hdRowD.size());
  d.hcG = c->dalloc<int>((int64_t)hdRowD.size());
  d.hcCp = c->dalloc<int>((int64_t)hdRowD.size());
  d.hcCf = c->dalloc<int64_t>((int64_t)hdRowD.size());
  d.hcStride = c->dalloc<int>((int64_t)hdRowD.size());
  d.hcColSlot = c->dalloc<int>((int64_t)hColSlot.size());
  d.hcColD = c->dalloc<int>((int64_t)hColSlot.size());
  d.hcColAtom = c->dalloc<int>((int64_t)hColSlot.size());
  d.Zbuf = nullptr;
  c->n_z = zOff[ntri];
  std::vector<int64_t> yOff(nCp + 1, 0);
  for (int i = 0; i < nCp; ++i) yOff[i + 1] = yOff[i] + (cfOff[i + 1] - cfOff[i]) * c->nsplit[i];
  d.yOff = c->upload(yOff);
  d.Ybuf = nullptr;
  c->n_y = yOff[nCp];
  c->have_f32 = c->have_f64 = false;
  d.Cf32 = nullptr; d.Vf32 = nullptr; d.D32 = nullptr; d.H32 = nullptr; d.Zbuf32 = nullptr; d.Ybuf32 = nullptr;
  d.gC = c->dalloc<double>(3 * c->nC);
  d.gV = c->dalloc<double>(3 * c->nV);
  d.Ep = c->dalloc<double>(nVp);
  d.atCfRow = c->upload(atCfRow); d.atCf = c->upload(atCf);
  d.atCsRow = c->upload(atCsRow); d.atCs = c->upload(atCs);
  d.atVfRow = c->upload(atVfRow); d.atVf = c->upload(atVf);
  d.atVsRow = c->upload(atVsRow); d.atVs = c->upload(atVs);
  d.out = c->dalloc<double>(1 + 3 * N + 9);
  d.err = c->dalloc<int>(1);
  g_pinned.put(c->h_out, c->h_out_bytes);
  c->h_out = nullptr;
  c->h_out_bytes = sizeof(double) * (1 + 3 * N + 9);
  c->h_out = (double*)g_pinned.get(c->h_out_bytes);

  // ---- value validation on the device ------------------------------------
  HIPCHK(hipMemsetAsync(d.err, 0, sizeof(int), c->stream));
  lrx::launch_validate_finite(d.Cval, C->nval, d.err, 1, c->stream);
  lrx::launch_validate_finite(d.Cdval, 3 * C->nval, d.err, 1, c->stream);
  // V and dV: finiteness is checked by the mirror pass of launch_validate
  lrx::launch_validate(d, c->stream);
  if (!km) {
    lrx::launch_validate_dsym(d.D, ntot, 0, d.err, c->stream);
  } else {   // D(-R) = D(R)^H
    lrx::launch_validate_herm(d.D, d.DnIm, km->nk, d.dld, d.err, c->stream);
    if (d.DnIm) lrx::launch_validate_finite(d.DnIm, d.dsize, d.err, 4, c->stream);
  }
  HIPCHK(hipGetLastError());
  int herr = 0;
  HIPCHK(hipMemcpyAsync(&herr, d.err, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  if (herr) {
    std::string m = "invalid tensor values:";
    if (herr & 1) m += " non-finite C/dC;";
    if (herr & 2) m += " non-finite V/dV;";
    if (herr & 4) m += " non-finite D;";
    if (herr & 8) m += " V(B,A,-R) != V(A,B,R)^T;";
    if (herr & 16) m += " dV(B,A,-R) != -dV(A,B,R)^T;";
    if (herr & 32) m += " on-site C block not symmetric in (a,f);";
    if (herr & 64) m += km ? " D(-R) != D(R)^H;" : " D not symmetric;";
    c->free_tensors();
    throw Fail{LRX_EINVAL, m};
  }
  c->have_tensors = true;
  c->gen = g_gen++;
}

// Back from a k-point supercell to the unit cell the caller set.
void restore_unit_cell(lrx_ctx* c) {
  c->N = c->N0;
  c->tau = c->tau0;
  c->lat = c->lat0;
  c->nao = c->nao0;
  c->nabf = c->nabf0;
  c->ao = c->ao0;
  c->bvk = false;
}

}  // namespace

// ===========================================================================
extern "C" {

int lrx_create(lrx_ctx** out, int32_t device, void* hip_stream) {
  if (!out) return LRX_EINVAL;
  lrx_ctx* c = new (std::nothrow) lrx_ctx();
  if (!c) return LRX_ENOMEM;
  c->device = device;
  int rc = guarded(c, [&] {
    int n = 0;
    HIPCHK(hipGetDeviceCount(&n));
    require(device >= 0 && device < n, "no such HIP device");
    if (hip_stream) {
      c->stream = (hipStream_t)hip_stream;
    } else {
      c->stream = g_streams.get(device);
      c->own_stream = true;
    }
    for (auto& e : c->ev) HIPCHK(hipEventCreate(&e));
    for (auto& e : c->gev) HIPCHK(hipEventCreate(&e));
    for (auto& e : c->fork) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->events = true;
    for (auto& st : c->side) st = g_streams.get(device);
    c->scratch = scratch_on(device);
  });
  if (rc != LRX_OK) {
    lrx_destroy(c);
    return rc;
  }
  *out = c;
  return LRX_OK;
}

int lrx_set_structure(lrx_ctx* c, int32_t natom, const double* tau, const double* lattice, const int32_t* nao,
                      const int32_t* nabf) {
  return guarded(c, [&] {
    require(natom > 0 && tau && lattice && nao && nabf, "lrx_set_structure: bad arguments");
    drop_plans_of(c);
    c->free_tensors();
    c->have_structure = false;
    c->bvk = false;
    c->N = natom;
    c->tau.assign(tau, tau + 3 * natom);
    c->lat.assign(lattice, lattice + 9);
    c->nao.assign(nao, nao + natom);
    c->nabf.assign(nabf, nabf + natom);
    c->ao.assign(natom + 1, 0);
    for (int i = 0; i < natom; ++i) {
      require(nao[i] >= 1 && nao[i] <= lrx::kMaxNao, "nao out of range 1..32");
      require(nabf[i] >= 1 && nabf[i] <= lrx::kMaxNabf, "nabf out of range 1..128");
      c->ao[i + 1] = c->ao[i] + nao[i];
    }
    for (double v : c->tau) require(std::isfinite(v), "non-finite position");
    const double* L = lattice;
    c->omega = std::fabs(L[0] * (L[4] * L[8] - L[5] * L[7]) - L[1] * (L[3] * L[8] - L[5] * L[6]) +
                         L[2] * (L[3] * L[7] - L[4] * L[6]));
    require(c->omega > 0 && std::isfinite(c->omega), "singular lattice");
    c->have_structure = true;
  });
}

int lrx_set_tensors(lrx_ctx* c, const lrx_blocks* C, const lrx_blocks* V, const double* D, int32_t on_device) {
  return guarded(c, [&] {
    require(c->have_structure, "lrx_set_tensors before lrx_set_structure");
    drop_plans_of(c);
    c->free_tensors();
    if (c->bvk) restore_unit_cell(c);
    check_blocks(c, C, true, "C");
    check_blocks(c, V, false, "V");
    require(D != nullptr, "D: NULL");
    build_tensors(c, C, V, D, on_device != 0, on_device != 0, nullptr);
  });
}

int lrx_set_kpoint_tensors(lrx_ctx* c, const int32_t* nk, const lrx_blocks* C, const lrx_blocks* V,
                           const double* Dre, const double* Dim, int32_t on_device) {
  return guarded(c, [&] {
    require(c->have_structure, "lrx_set_kpoint_tensors before lrx_set_structure");
    require(nk != nullptr && Dre != nullptr, "lrx_set_kpoint_tensors: NULL argument");
    drop_plans_of(c);
    c->free_tensors();
    if (c->bvk) restore_unit_cell(c);
    for (int x = 0; x < 3; ++x) require(nk[x] >= 1 && nk[x] <= 64, "nk out of range 1..64");
    const int ncell = nk[0] * nk[1] * nk[2];
    const int N0 = c->N;
    require((int64_t)N0 * ncell <= 16384, "k-point supercell of more than 16384 atoms");
    require(ncell < 1024, "k mesh of 1024 points or more");
    require(c->ao[N0] < (1 << 21), "more than 2097151 NAOs in the unit cell");
    check_blocks(c, C, true, "C");   // the caller's keys, on the unit cell
    check_blocks(c, V, false, "V");
    const int64_t nt0 = c->ao[N0];
    // keys on the supercell: (A, F, R) -> (A, (R mod nk, F), (R - R mod nk) / nk)
    KMap km;
    km.N0 = N0;
    for (int x = 0; x < 3; ++x) km.nk[x] = nk[x];
    km.VR0 = V->R;
    std::vector<int32_t> cS, cR, vS, vR;
    auto convert = [&](const lrx_blocks* B, std::vector<int32_t>& S, std::vector<int32_t>& R) {
      S.resize(B->nblk);
      R.resize(3 * B->nblk);
      for (int64_t b = 0; b < B->nblk; ++b) {
        int r[3];
        for (int x = 0; x < 3; ++x) {
          const int v = B->R[3 * b + x];
          r[x] = ((v % nk[x]) + nk[x]) % nk[x];
          R[3 * b + x] = (v - r[x]) / nk[x];
        }
        S[b] = (r[0] + nk[0] * (r[1] + nk[1] * r[2])) * N0 + B->second[b];
      }
    };
    convert(C, cS, cR);
    convert(V, vS, vR);
    lrx_blocks C2 = *C, V2 = *V;
    C2.second = cS.data();
    C2.R = cR.data();
    V2.second = vS.data();
    V2.R = vR.data();
    // the unit cell is kept; the context describes the supercell (the volume
    // stays the unit cell's: the stress per unit cell)
    c->N0 = N0;
    c->tau0 = c->tau;
    c->lat0 = c->lat;
    c->nao0 = c->nao;
    c->nabf0 = c->nabf;
    c->ao0 = c->ao;
    for (int x = 0; x < 3; ++x) c->nk[x] = nk[x];
    const int Ns = N0 * ncell;
    c->N = Ns;
    c->tau.assign(3 * (size_t)Ns, 0.0);
    c->nao.assign(Ns, 0);
    c->nabf.assign(Ns, 0);
    for (int t = 0; t < ncell; ++t) {
      const int t0 = t % nk[0], t1 = (t / nk[0]) % nk[1], t2 = t / (nk[0] * nk[1]);
      for (int i = 0; i < N0; ++i) {
        for (int x = 0; x < 3; ++x)
          c->tau[3 * ((size_t)t * N0 + i) + x] =
              c->tau0[3 * i + x] + t0 * c->lat0[x] + t1 * c->lat0[3 + x] + t2 * c->lat0[6 + x];
        c->nao[t * N0 + i] = c->nao0[i];
        c->nabf[t * N0 + i] = c->nabf0[i];
      }
    }
    for (int r = 0; r < 3; ++r)
      for (int x = 0; x < 3; ++x) c->lat[3 * r + x] = nk[r] * c->lat0[3 * r + x];
    c->ao.assign(Ns + 1, 0);
    for (int i = 0; i < Ns; ++i) c->ao[i + 1] = c->ao[i] + c->nao[i];
    c->bvk = true;
    // D(R) on the device, read where it is (the block of two supercell atoms is
    // that of their cells' offset): device arrays are borrowed, host arrays copied
    auto to_device = [&](const double* Dk) -> const double* {
      if (on_device) return Dk;
      double* p = c->dalloc<double>((int64_t)ncell * nt0 * nt0);
      HIPCHK(hipMemcpyAsync(p, Dk, sizeof(double) * ncell * nt0 * nt0, hipMemcpyHostToDevice, c->stream));
      return p;
    };
    const double* DkRe = to_device(Dre);
    const double* DkIm = Dim ? to_device(Dim) : nullptr;
    km.Dim = DkIm;
    build_tensors(c, &C2, &V2, DkRe, true, on_device != 0, &km);
    c->DscIm = DkIm;
  });
}

}  // extern "C"

namespace {

// The screening options of a call.
lrx::Opts make_opts(const lrx_options* o) {
  lrx::Opts r{o->theta, o->theta_cs, o->precision};
  r.per_tensor = (o->flags & LRX_SCREEN_PER_TENSOR) != 0;
  for (int k = 0; k < 5; ++k) r.th[k] = o->theta_tensor[k];
  return r;
}

// Checks shared by lrx_evaluate and lrx_evaluate_batch; allocates the FP32
// buffers of a reduced-precision form on first use.
void prepare(lrx_ctx* c, const lrx_options* opts) {
  require(opts != nullptr, "opts: NULL");
  require(c->have_tensors, "evaluation before lrx_set_tensors");
  require(opts->precision == LRX_FP64 || opts->precision == LRX_FP32 || opts->precision == LRX_BF16X3,
          "unknown precision");
  require(std::isfinite(opts->theta) && std::isfinite(opts->theta_cs), "non-finite threshold");
  if (opts->flags & LRX_SCREEN_PER_TENSOR)
    for (int k = 0; k < 5; ++k) require(std::isfinite(opts->theta_tensor[k]), "non-finite threshold");
  c->per_tensor = (opts->flags & LRX_SCREEN_PER_TENSOR) != 0;
  if (opts->precision == LRX_FP64 && !c->have_f64) {
    Dev& d = c->dev;
    d.H = c->dalloc<double>(c->n_h);
    HIPCHK(hipMemsetAsync(d.H, 0, sizeof(double) * std::max<int64_t>(1, c->n_h), c->stream));   // zero padding rows
    d.Zbuf = c->dalloc<double>(c->n_z);
    d.Ybuf = c->dalloc<double>(c->n_y);
    c->have_f64 = true;
    c->gen = g_gen++;
  }
  if (opts->precision != LRX_FP64 && !c->have_f32) {
    Dev& d = c->dev;
    const int64_t nt = c->ao[c->N];
    d.Cf32 = c->dalloc<float>(c->n_cf);
    d.Vf32 = c->dalloc<float>(c->n_vf);
    d.D32 = c->dalloc<float>(d.dsize);
    d.H32 = c->dalloc<float>(c->n_h);
    HIPCHK(hipMemsetAsync(d.H32, 0, sizeof(float) * std::max<int64_t>(1, c->n_h), c->stream));
    d.Zbuf32 = c->dalloc<float>(c->n_z);
    d.Ybuf32 = c->dalloc<float>(c->n_y);
    c->have_f32 = true;
    c->gen = g_gen++;
  }
}

// One evaluation with k-point sampling: the screening and contraction kernels
// on the supercell (home-cell rows), once with the real part of D and, for a
// complex D, once more with its imaginary part.  The kernels weigh a quartet
// with M_AB M_GF + M_FB M_GA (H(B,X) reads the rows G of M).  For a
// Hermitian D, Re[D_AB D*_FG + D_AG D*_FB] is that weight of the symmetric
// real part minus that weight of the antisymmetric imaginary part, so E, F,
// sigma and the block gradients are the first pass minus the second.  Both
// passes keep the same blocks: C and V are real, and the D screen measures
// the modulus.
void bvk_evaluate(lrx_ctx* c, const lrx_options* opts, double* E, double* F, double* sigma) {
  prepare(c, opts);
  require(!(opts->theta_cs > 0), "k-point sampling: step 2 (theta_cs > 0) is not available");
  const lrx::Opts o = make_opts(opts);
  const int64_t nout = 1 + 3 * (int64_t)c->N + 9;
  for (int mt = 0; mt <= lrx::kMaxAlphaTiles; ++mt) c->tl.mode[mt] = 1;
  Dev d = c->dev;
  const int passes = c->DscIm ? 2 : 1;
  if (passes == 2 && !c->keep2) c->keep2 = c->dalloc<double>(3 * c->nC + 3 * c->nV + nout);
  for (int pass = 0; pass < passes; ++pass) {
    if (pass == 1) {
      if (c->nC)
        HIPCHK(hipMemcpyAsync(c->keep2, d.gC, sizeof(double) * 3 * c->nC, hipMemcpyDeviceToDevice, c->stream));
      if (c->nV)
        HIPCHK(hipMemcpyAsync(c->keep2 + 3 * c->nC, d.gV, sizeof(double) * 3 * c->nV, hipMemcpyDeviceToDevice,
                              c->stream));
      HIPCHK(hipMemcpyAsync(c->keep2 + 3 * c->nC + 3 * c->nV, d.out, sizeof(double) * nout,
                            hipMemcpyDeviceToDevice, c->stream));
      d.D = c->DscIm;
    }
    // the second pass keeps every decision, list and folded block of the
    // first (they do not depend on D's values beyond the modulus the D
    // screen measured); only D's FP32 copy changes
    if (pass == 0)
      lrx::launch_screen(d, o, c->stream, nullptr);
    else
      lrx::launch_d_to_f32(d, opts->precision, c->stream);
    c->tl.devs.s[0] = d;
    lrx::launch_contract(d, c->tl, opts->precision, c->stream, c->side.data(), c->fork.data(), nullptr, nullptr);
  }
  if (passes == 2) {
    lrx::launch_sub_from(c->keep2, d.gC, 3 * c->nC, c->stream);
    lrx::launch_sub_from(c->keep2 + 3 * c->nC, d.gV, 3 * c->nV, c->stream);
    lrx::launch_sub_from(c->keep2 + 3 * c->nC + 3 * c->nV, d.out, nout, c->stream);
  }
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->h_out, d.out, sizeof(double) * nout, hipMemcpyDeviceToHost, c->stream));
  HIPCHK(hipStreamSynchronize(c->stream));
  c->timed = false;
  c->evaluated = true;
  if (E) *E = c->h_out[0];
  if (F) std::memcpy(F, c->h_out + 1, sizeof(double) * 3 * c->N0);
  if (sigma) std::memcpy(sigma, c->h_out + 1 + 3 * c->N, sizeof(double) * 9);
}

}  // namespace

extern "C" {

int lrx_block_gradients(lrx_ctx* c, double* gC, double* gV) {
  return guarded(c, [&] {
    require(c->evaluated, "no evaluation yet");
    if (gC && c->nC) HIPCHK(hipMemcpyAsync(gC, c->dev.gC, sizeof(double) * 3 * c->nC, hipMemcpyDeviceToHost, c->stream));
    if (gV && c->nV) HIPCHK(hipMemcpyAsync(gV, c->dev.gV, sizeof(double) * 3 * c->nV, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  });
}

int lrx_keep_masks(lrx_ctx* c, uint8_t* keepC, uint8_t* keepV, uint8_t* keepD) {
  return guarded(c, [&] {
    require(c->evaluated, "no evaluation yet");
    if (keepC && c->nC) HIPCHK(hipMemcpyAsync(keepC, c->dev.keepC, c->nC, hipMemcpyDeviceToHost, c->stream));
    if (keepV && c->nV) HIPCHK(hipMemcpyAsync(keepV, c->dev.keepV, c->nV, hipMemcpyDeviceToHost, c->stream));
    if (keepD) HIPCHK(hipMemcpyAsync(keepD, c->dev.keepD, (size_t)c->N * c->N, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (!c->per_tensor) {   // the joint lists: 0/1 per block
      if (keepC)
        for (int64_t b = 0; b < c->nC; ++b) keepC[b] = keepC[b] != 0;
      if (keepV)
        for (int64_t b = 0; b < c->nV; ++b) keepV[b] = keepV[b] != 0;
    }
  });
}

int lrx_get_stats(lrx_ctx* c, lrx_stats* s) {
  return guarded(c, [&] {
    require(s != nullptr, "NULL stats");
    require(c->have_tensors, "no tensors yet");
    auto work = [&](lrx_stats* o) {
      const int64_t nt = c->ao[c->N];
      o->work_bytes[LRX_FP64] = 8.0 * (double)(c->n_h + c->n_z + c->n_y);
      o->work_bytes[LRX_FP32] = 4.0 * (double)(c->n_cf + c->n_vf + nt * nt + c->n_h + c->n_z + c->n_y);
      o->work_bytes[LRX_BF16X3] = o->work_bytes[LRX_FP32];
      o->work_held[LRX_FP64] = c->have_f64;
      o->work_held[LRX_FP32] = o->work_held[LRX_BF16X3] = c->have_f32;
      o->device_bytes = c->dev_bytes;
    };
    if (!c->evaluated) {   // before the first evaluation only the memory is known
      *s = lrx_stats{};
      work(s);
      return;
    }
    const Dev& d = c->dev;
    std::vector<uint8_t> kC(c->nC), kV(c->nV), aC(d.nCp), aV(d.nVp), need(d.nSlot);
    if (c->nC) HIPCHK(hipMemcpyAsync(kC.data(), d.keepC, c->nC, hipMemcpyDeviceToHost, c->stream));
    if (c->nV) HIPCHK(hipMemcpyAsync(kV.data(), d.keepV, c->nV, hipMemcpyDeviceToHost, c->stream));
    if (d.nCp) HIPCHK(hipMemcpyAsync(aC.data(), d.aliveC, d.nCp, hipMemcpyDeviceToHost, c->stream));
    if (d.nVp) HIPCHK(hipMemcpyAsync(aV.data(), d.aliveV, d.nVp, hipMemcpyDeviceToHost, c->stream));
    if (d.nSlot) HIPCHK(hipMemcpyAsync(need.data(), d.need, d.nSlot, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    *s = lrx_stats{};
    const auto& na = c->nao;
    const auto& nb = c->nabf;
    double fl = 0, ft = 0, by = 0;
    for (int64_t b = 0; b < c->nC; ++b) {
      const double sz = (double)nb[c->Cf[b]] * na[c->Cf[b]] * na[c->Cs[b]];
      by += 4 * sz * 8;
      if (kC[b]) { s->kept_c_blocks++; fl += 6 * sz; }
    }
    for (int64_t b = 0; b < c->nV; ++b) {
      const double sz = (double)nb[c->Vf[b]] * nb[c->Vs[b]];
      by += 4 * sz * 8;
      if (kV[b]) { s->kept_v_blocks++; fl += 8 * sz; }
    }
    by += (double)c->ao[c->N] * c->ao[c->N] * 8;
    for (int i = 0; i < d.nCp; ++i) s->alive_c_pairs += aC[i] != 0;
    for (int i = 0; i < d.nVp; ++i) s->alive_v_pairs += aV[i] != 0;
    const Pairs& cp = c->cp;
    const Pairs& vp = c->vp;
    for (int i = 0; i < d.nCp; ++i) {
      if (!aC[i]) continue;
      const int A = cp.pA[i], Fa = cp.pB[i];
      for (int p = vp.row[A]; p < vp.row[A + 1]; ++p) {
        const int B = vp.pB[p];
        if (!lrx::triple_live(aC[i], aV[p], !c->vpZown[p])) continue;
        s->alive_triples++;
        // Y and (when this unit forms it: the pair forms Z and Cf(A,F) is
        // live; the mirror's Z is the transpose) Z, and the X-build
        const double zy = lrx::unit_y_only(aC[i], !c->vpZown[p]) ? 2.0 : 4.0;
        const double t = zy * nb[A] * nb[B] * na[A] * na[Fa] + 4.0 * nb[B] * na[A] * na[B] * na[Fa];
        ft += t;
        s->flop_triple_group[(nb[A] + 15) / 16] += t;
      }
    }
    for (int sl = 0; sl < d.nSlot; ++sl) {
      if (!need[sl]) continue;
      s->h_slots++;
      const int B = c->slotB[sl], X = c->slotX[sl];
      double depth = 0;
      for (int i = cp.row[B]; i < cp.row[B + 1]; ++i)
        if (aC[i] & 1) depth += na[cp.pB[i]];
      fl += 2.0 * nb[B] * na[B] * na[X] * depth;
    }
    s->flop_triple = ft;
    s->flop_alg = fl + ft;
    s->bytes_alg = by;
    work(s);
  });
}

int lrx_group_times(lrx_ctx* c, float* ms, int32_t n) {
  if (!c) return LRX_EINVAL;
  if (!c->timed) {
    c->err = "no timed evaluation yet";
    return LRX_ESTATE;
  }
  for (int i = 0; i < n && i <= lrx::kMaxAlphaTiles; ++i) ms[i] = c->group_ms[i];
  return lrx::kMaxAlphaTiles + 1;
}

int lrx_stage_times(lrx_ctx* c, float* ms, int32_t n) {
  if (!c) return LRX_EINVAL;
  if (!c->timed) {
    c->err = "no timed evaluation yet";
    return LRX_ESTATE;
  }
  for (int i = 0; i < n && i < LRX_NSTAGES; ++i) ms[i] = c->stage_ms[i];
  return LRX_NSTAGES;
}

const char* lrx_stage_name(int32_t i) {
  static const char* names[LRX_NSTAGES] = {"norms", "screen", "fold", "mark", "hbuild",
                                           "triple", "zgrad", "cgrad", "forces"};
  return (i >= 0 && i < LRX_NSTAGES) ? names[i] : "";
}

}  // extern "C"

namespace {

// A batch of structures evaluated together: the screening, folding, H-build
// and gradient kernels of every structure and, per alpha-tile group, one
// triple launch per kBatchDevs structures whose work items interleave the
// structures' units.  Built once per (contexts, options); the launch shape of
// every group is picked by timing (autotuner), and the whole kernel sequence
// is captured in a HIP graph that later calls replay.
struct BatchPlan {
  int device = 0;
  std::vector<lrx_ctx*> ctxs;
  std::vector<uint64_t> gens;
  int prec = 0, flags = 0;
  double theta = 0, theta_cs = 0;
  lrx::Opts opts{};
  std::vector<lrx::TripleLaunch> launches;
  std::vector<void*> allocs;
  hipStream_t stream = nullptr;   // the first context's stream
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int uses = 0;
  std::array<int, lrx::kMaxAlphaTiles + 1> mode{};
  std::array<float, 2 * (lrx::kMaxAlphaTiles + 1)> tune_ms{};

  ~BatchPlan() {
    (void)hipSetDevice(device);
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    // after the plan's last launch on its stream (every context of a plan,
    // and so its stream, outlives the plan)
    (void)hipStreamSynchronize(stream);
    for (void* p : allocs) lrx::dev_free(device, p);
  }
  bool matches(lrx_ctx* const* c, int n, const lrx_options* o) const {
    if ((int)ctxs.size() != n || prec != o->precision || theta != o->theta || theta_cs != o->theta_cs ||
        flags != o->flags)
      return false;
    for (int k = 0; k < 5; ++k)
      if ((flags & LRX_SCREEN_PER_TENSOR) && opts.th[k] != o->theta_tensor[k]) return false;
    for (int i = 0; i < n; ++i)
      if (ctxs[i] != c[i] || gens[i] != c[i]->gen) return false;
    return true;
  }
  template <class T>
  T* upload(const std::vector<T>& v, hipStream_t s) {
    void* p = nullptr;
    p = lrx::dev_alloc(device, std::max<size_t>(1, v.size() * sizeof(T)));
    if (!p) throw Fail{LRX_ENOMEM, "device memory exhausted (batch plan)"};
    stream = s;
    allocs.push_back(p);
    if (!v.empty()) HIPCHK(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s));
    return (T*)p;
  }
};

std::mutex g_plan_mu;
std::vector<std::shared_ptr<BatchPlan>> g_plans;   // most recently used last
constexpr size_t kMaxPlans = 8;
// launch shape chosen by the autotuner per (precision, alpha group), -1 until
// a plan has timed that group; later plans take it without timing again
std::array<std::array<int, lrx::kMaxAlphaTiles + 1>, 3> g_tuned = [] {
  std::array<std::array<int, lrx::kMaxAlphaTiles + 1>, 3> t{};
  for (auto& r : t) r.fill(-1);
  return t;
}();

void drop_plans_of(const lrx_ctx* c) {
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plans.erase(std::remove_if(g_plans.begin(), g_plans.end(),
                               [&](const std::shared_ptr<BatchPlan>& p) {
                                 return std::find(p->ctxs.begin(), p->ctxs.end(), c) != p->ctxs.end();
                               }),
                g_plans.end());
}

// Alpha-tile groups of a plan, largest first.
std::vector<int> group_order(const BatchPlan& P) {
  std::vector<int> order;
  std::array<long, lrx::kMaxAlphaTiles + 1> tot{};
  for (const auto& L : P.launches)
    for (int mt = 1; mt <= lrx::kMaxAlphaTiles; ++mt) tot[mt] += L.n[mt];
  for (int mt = 1; mt <= lrx::kMaxAlphaTiles; ++mt)
    if (tot[mt] > 0) order.push_back(mt);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return tot[a] > tot[b]; });
  return order;
}

// Every kernel of one batched evaluation, on stream s (side streams carry the
// smaller alpha-tile groups and join back before the gradients).
void run_batch(const BatchPlan& P, hipStream_t s, const hipStream_t* side, const hipEvent_t* fork) {
  const lrx::Opts o = P.opts;
  for (lrx_ctx* c : P.ctxs) lrx::launch_screen(c->dev, o, s, nullptr);
  for (lrx_ctx* c : P.ctxs) lrx::launch_hbuild(c->dev, P.prec, s);
  const std::vector<int> order = group_order(P);
  (void)hipEventRecord(fork[0], s);
  for (size_t i = 0; i < order.size(); ++i) {
    const hipStream_t st = i == 0 ? s : side[(i - 1) % lrx::kSideStreams];
    if (i > 0 && i <= (size_t)lrx::kSideStreams) (void)hipStreamWaitEvent(st, fork[0], 0);
    for (const auto& L : P.launches) lrx::launch_triple_group(L, order[i], P.prec, st);
  }
  for (size_t i = 1; i <= (size_t)lrx::kSideStreams && i < order.size(); ++i) {
    (void)hipEventRecord(fork[i], side[i - 1]);
    (void)hipStreamWaitEvent(s, fork[i], 0);
  }
  for (lrx_ctx* c : P.ctxs) lrx::launch_grads(c->dev, P.prec, s, nullptr);
}

std::shared_ptr<BatchPlan> build_plan(lrx_ctx* const* ctxs, int n, const lrx_options* opts) {
  lrx_ctx* c0 = ctxs[0];
  auto P = std::make_shared<BatchPlan>();
  P->device = c0->device;
  P->ctxs.assign(ctxs, ctxs + n);
  for (int i = 0; i < n; ++i) P->gens.push_back(ctxs[i]->gen);
  P->prec = opts->precision;
  P->flags = opts->flags;
  P->theta = opts->theta;
  P->theta_cs = opts->theta_cs;
  P->opts = make_opts(opts);
  for (int g0 = 0; g0 < n; g0 += lrx::kBatchDevs) {
    lrx::TripleLaunch L{};
    const int ng = std::min(lrx::kBatchDevs, n - g0);
    for (int j = 0; j < ng; ++j) L.devs.s[j] = ctxs[g0 + j]->dev;
    std::vector<int2> items;
    std::array<int, lrx::kMaxAlphaTiles + 2> start{};
    for (int mt = 1; mt <= lrx::kMaxAlphaTiles; ++mt) {
      start[mt] = (int)items.size();
      // the structures' units of this group, interleaved in blocks so each
      // structure's neighbouring units still land on the same XCD
      std::vector<size_t> pos(ng, 0);
      bool more = true;
      while (more) {
        more = false;
        for (int j = 0; j < ng; ++j) {
          const lrx_ctx* c = ctxs[g0 + j];
          const int a = c->mtStartHost[mt], b = c->mtStartHost[mt + 1];
          for (int k = 0; k < 64 && a + (int)pos[j] < b; ++k, ++pos[j])
            items.push_back(make_int2(j, c->unitOrderHost[a + pos[j]]));
          if (a + (int)pos[j] < b) more = true;
        }
      }
      start[mt + 1] = (int)items.size();
    }
    int2* it = P->upload(items, c0->stream);
    for (int mt = 1; mt <= lrx::kMaxAlphaTiles; ++mt) {
      L.items[mt] = it + start[mt];
      L.n[mt] = start[mt + 1] - start[mt];
    }
    L.counters = P->upload(std::vector<int>(8 * (lrx::kMaxAlphaTiles + 1), 0), c0->stream);
    P->launches.push_back(L);
  }
  hipStream_t s = c0->stream;
  // shapes already tuned in this process are reused; without the tuner a
  // group takes the persistent grid, the shape the tuner has preferred on
  // every workload measured so far
  std::vector<int> to_tune;
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (int mt = 0; mt <= lrx::kMaxAlphaTiles; ++mt) {
      const int t = g_tuned[P->prec][mt];
      P->mode[mt] = t >= 0 ? t : 1;
    }
    for (int mt : group_order(*P))
      if (g_tuned[P->prec][mt] < 0) to_tune.push_back(mt);
  }
  for (auto& L : P->launches)
    for (int mt = 0; mt <= lrx::kMaxAlphaTiles; ++mt) L.mode[mt] = P->mode[mt];
  if (!(opts->flags & LRX_BATCH_NO_TUNE) && !to_tune.empty()) {
    // warm-up run: fills every intermediate buffer and sets kernel attributes
    run_batch(*P, s, c0->side.data(), c0->fork.data());
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s));
    // autotuner: per alpha-tile group, one workgroup per item (mode 0) or a
    // persistent grid (mode 1), best of two timed launches of the group alone
    // (the triple kernels only overwrite their own partial sums, so repeating
    // them is harmless)
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    for (int mt : to_tune) {
      float best[2] = {1e30f, 1e30f};
      for (int mode = 0; mode < 2; ++mode) {
        for (auto& L : P->launches) L.mode[mt] = mode;
        for (int rep = 0; rep < 2; ++rep) {
          HIPCHK(hipEventRecord(e0, s));
          for (const auto& L : P->launches) lrx::launch_triple_group(L, mt, P->prec, s);
          HIPCHK(hipEventRecord(e1, s));
          HIPCHK(hipEventSynchronize(e1));
          float ms = 0;
          HIPCHK(hipEventElapsedTime(&ms, e0, e1));
          best[mode] = std::min(best[mode], ms);
        }
      }
      P->mode[mt] = best[1] < best[0] ? 1 : 0;
      P->tune_ms[2 * mt] = best[0];
      P->tune_ms[2 * mt + 1] = best[1];
      for (auto& L : P->launches) L.mode[mt] = P->mode[mt];
      std::lock_guard<std::mutex> lk(g_plan_mu);
      g_tuned[P->prec][mt] = P->mode[mt];
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  c0->tune_mode = P->mode;
  c0->tune_ms = P->tune_ms;
  return P;
}

// Run a plan on the first context's stream: eagerly on its first use, then
// from the HIP graph captured on its second use (a plan used once, e.g. a
// one-off batch, never pays for a capture).  The legacy default stream cannot
// be captured: such contexts, and plans asked to run eagerly, stay eager.
void launch_plan(BatchPlan& P, const lrx_options* opts) {
  lrx_ctx* c0 = P.ctxs[0];
  hipStream_t s = c0->stream;
  ++P.uses;
  const bool capturable = s != nullptr && !(opts->flags & LRX_BATCH_EAGER);
  if (capturable && !P.exec && P.uses >= 2) {
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    run_batch(P, s, c0->side.data(), c0->fork.data());
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamEndCapture(s, &g));
    P.graph = g;
    HIPCHK(hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0));
  }
  if (capturable && P.exec)
    HIPCHK(hipGraphLaunch(P.exec, s));
  else
    run_batch(P, s, c0->side.data(), c0->fork.data());
}

// The plan of (contexts, options): from the cache, or built (and cached).
std::shared_ptr<BatchPlan> get_plan(lrx_ctx* const* ctxs, int n, const lrx_options* opts) {
  {
    std::lock_guard<std::mutex> lk(g_plan_mu);
    for (size_t k = 0; k < g_plans.size(); ++k)
      if (g_plans[k]->matches(ctxs, n, opts)) {
        std::shared_ptr<BatchPlan> P = g_plans[k];
        g_plans.erase(g_plans.begin() + k);
        g_plans.push_back(P);
        return P;
      }
  }
  std::shared_ptr<BatchPlan> P = build_plan(ctxs, n, opts);
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plans.push_back(P);
  if (g_plans.size() > kMaxPlans) g_plans.erase(g_plans.begin());
  return P;
}

}  // namespace

extern "C" {

int lrx_evaluate(lrx_ctx* c, const lrx_options* opts, double* E, double* F, double* sigma) {
  return guarded(c, [&] {
    if (c->bvk) {
      bvk_evaluate(c, opts, E, F, sigma);
      return;
    }
    prepare(c, opts);
    lrx_ctx* one[1] = {c};
    // launch shapes from the autotuner; the captured graph unless stage
    // times are requested
    std::shared_ptr<BatchPlan> P = get_plan(one, 1, opts);
    const bool timing = opts->timing != 0;
    if (timing) {
      const lrx::Opts o = make_opts(opts);
      hipEvent_t* ev = timing ? c->ev.data() + 1 : nullptr;
      if (timing) HIPCHK(hipEventRecord(c->ev[0], c->stream));
      lrx::launch_screen(c->dev, o, c->stream, ev);
      c->tl.devs.s[0] = c->dev;
      for (int mt = 0; mt <= lrx::kMaxAlphaTiles; ++mt) c->tl.mode[mt] = P->mode[mt];
      lrx::launch_contract(c->dev, c->tl, opts->precision, c->stream, c->side.data(), c->fork.data(), ev,
                           c->gev.data());
    } else {
      launch_plan(*P, opts);
    }
    HIPCHK(hipGetLastError());
    const int N = c->N;
    HIPCHK(hipMemcpyAsync(c->h_out, c->dev.out, sizeof(double) * (1 + 3 * N + 9), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (timing) {
      for (int i = 0; i < LRX_NSTAGES; ++i) HIPCHK(hipEventElapsedTime(&c->stage_ms[i], c->ev[i], c->ev[i + 1]));
      for (int mt = 0; mt <= lrx::kMaxAlphaTiles; ++mt) {
        c->group_ms[mt] = 0.f;
        if (c->tl.n[mt] > 0) HIPCHK(hipEventElapsedTime(&c->group_ms[mt], c->gev[2 * mt], c->gev[2 * mt + 1]));
      }
    }
    c->timed = timing;
    c->evaluated = true;
    if (E) *E = c->h_out[0];
    if (F) std::memcpy(F, c->h_out + 1, sizeof(double) * 3 * N);
    if (sigma) std::memcpy(sigma, c->h_out + 1 + 3 * N, sizeof(double) * 9);
  });
}

int lrx_submit(lrx_ctx* c, const lrx_options* opts, int64_t* ticket) {
  return guarded(c, [&] {
    require(ticket != nullptr, "ticket: NULL");
    require(!c->bvk, "lrx_submit: k-point contexts are evaluated with lrx_evaluate");
    require(opts != nullptr, "opts: NULL");
    require(opts->timing == 0, "lrx_submit: stage times need lrx_evaluate");
    prepare(c, opts);
    lrx_ctx* one[1] = {c};
    std::shared_ptr<BatchPlan> P = get_plan(one, 1, opts);
    launch_plan(*P, opts);
    HIPCHK(hipGetLastError());
    lrx_ctx::Ticket t;
    t.N = c->N;
    t.bytes = sizeof(double) * (1 + 3 * c->N + 9);
    HIPCHK(hipEventCreateWithFlags(&t.done, hipEventDisableTiming));
    try {
      t.h = (double*)g_pinned.get(t.bytes);
      // the next evaluation on this stream overwrites dev.out only after this copy
      HIPCHK(hipMemcpyAsync(t.h, c->dev.out, t.bytes, hipMemcpyDeviceToHost, c->stream));
      HIPCHK(hipEventRecord(t.done, c->stream));
    } catch (...) {
      c->release(t);
      throw;
    }
    c->timed = false;
    c->evaluated = true;
    const int64_t id = c->next_ticket++;
    c->tickets[id] = t;
    *ticket = id;
  });
}

int lrx_wait(lrx_ctx* c, int64_t ticket, double* E, double* F, double* sigma) {
  return guarded(c, [&] {
    auto it = c->tickets.find(ticket);
    require(it != c->tickets.end(), "lrx_wait: unknown ticket (not submitted on this context, or already waited for)");
    lrx_ctx::Ticket t = it->second;
    c->tickets.erase(it);
    const hipError_t e = hipEventSynchronize(t.done);
    if (e == hipSuccess) {
      if (E) *E = t.h[0];
      if (F) std::memcpy(F, t.h + 1, sizeof(double) * 3 * t.N);
      if (sigma) std::memcpy(sigma, t.h + 1 + 3 * t.N, sizeof(double) * 9);
    }
    c->release(t);
    HIPCHK(e);
  });
}

int lrx_evaluate_batch(lrx_ctx* const* ctxs, int32_t n, const lrx_options* opts, double* E, double* F,
                       double* sigma) {
  if (!ctxs || n <= 0 || !ctxs[0]) return LRX_EINVAL;
  for (int i = 0; i < n; ++i)
    if (!ctxs[i]) return LRX_EINVAL;
  lrx_ctx* c0 = ctxs[0];
  return guarded(c0, [&] {
    for (int i = 0; i < n; ++i) {
      require(ctxs[i]->device == c0->device, "batch: contexts on different devices");
      require(!ctxs[i]->bvk, "batch: k-point contexts are evaluated with lrx_evaluate");
      for (int j = 0; j < i; ++j) require(ctxs[i] != ctxs[j], "batch: a context appears twice");
      prepare(ctxs[i], opts);
    }
    for (int i = 0; i < n; ++i)
      if (ctxs[i]->stream != c0->stream) HIPCHK(hipStreamSynchronize(ctxs[i]->stream));
    std::shared_ptr<BatchPlan> P = get_plan(ctxs, n, opts);
    hipStream_t s = c0->stream;
    launch_plan(*P, opts);
    HIPCHK(hipGetLastError());
    for (int i = 0; i < n; ++i) {
      lrx_ctx* c = ctxs[i];
      HIPCHK(hipMemcpyAsync(c->h_out, c->dev.out, sizeof(double) * (1 + 3 * c->N + 9), hipMemcpyDeviceToHost,
                            s));
    }
    HIPCHK(hipStreamSynchronize(s));
    int64_t fo = 0;
    for (int i = 0; i < n; ++i) {
      lrx_ctx* c = ctxs[i];
      c->evaluated = true;
      c->timed = false;
      if (E) E[i] = c->h_out[0];
      if (F) std::memcpy(F + fo, c->h_out + 1, sizeof(double) * 3 * c->N);
      if (sigma) std::memcpy(sigma + 9 * i, c->h_out + 1 + 3 * c->N, sizeof(double) * 9);
      fo += 3 * c->N;
    }
  });
}

int lrx_evaluate_noalloc(lrx_ctx* c, const lrx_options* opts, double* E, double* F, double* sigma) {
  return guarded(c, [&] {
    require(opts != nullptr, "opts: NULL");
    require(!c->bvk, "lrx_evaluate_noalloc: k-point contexts are evaluated with lrx_evaluate");
    require(c->have_tensors, "evaluation before lrx_set_tensors");
    const int prec = opts->precision;
    require(prec == LRX_FP64 || prec == LRX_FP32 || prec == LRX_BF16X3, "unknown precision");
    require(std::isfinite(opts->theta) && std::isfinite(opts->theta_cs), "non-finite threshold");
    if (opts->flags & LRX_SCREEN_PER_TENSOR)
      for (int k = 0; k < 5; ++k) require(std::isfinite(opts->theta_tensor[k]), "non-finite threshold");
    c->per_tensor = (opts->flags & LRX_SCREEN_PER_TENSOR) != 0;
    require(opts->timing == 0, "lrx_evaluate_noalloc: stage times need lrx_evaluate");
    require(c->scratch != nullptr, "lrx_evaluate_noalloc: no scratch address for this device");
    // the work buffers of this precision, carved from the scratch in 256-byte steps
    const int64_t nt = c->ao[c->N];
    auto al = [](size_t b) { return (std::max<size_t>(b, 1) + 255) & ~(size_t)255; };
    size_t need = 0;
    if (prec == LRX_FP64)
      need = al(8 * c->n_h) + al(8 * c->n_z) + al(8 * c->n_y);
    else
      need = al(4 * c->n_cf) + al(4 * c->n_vf) + al(4 * nt * nt) + al(4 * c->n_h) + al(4 * c->n_z) + al(4 * c->n_y);
    if (need > (size_t)LRX_SCRATCH_BYTES)
      throw Fail{LRX_EBUDGET, "lrx_evaluate_noalloc: this structure needs " + std::to_string(need) +
                                  " bytes of scratch, more than the fixed " + std::to_string((size_t)LRX_SCRATCH_BYTES)};
    Dev d = c->dev;
    size_t used = 0;
    auto carve = [&](size_t bytes) {
      unsigned char* p = c->scratch + used;
      used += al(bytes);
      return p;
    };
    unsigned char* hbase;
    size_t hbytes;
    if (prec == LRX_FP64) {
      d.H = (double*)(hbase = carve(hbytes = 8 * c->n_h));
      d.Zbuf = (double*)carve(8 * c->n_z);
      d.Ybuf = (double*)carve(8 * c->n_y);
    } else {
      d.Cf32 = (float*)carve(4 * c->n_cf);
      d.Vf32 = (float*)carve(4 * c->n_vf);
      d.D32 = (float*)carve(4 * nt * nt);
      d.H32 = (float*)(hbase = carve(hbytes = 4 * c->n_h));
      d.Zbuf32 = (float*)carve(4 * c->n_z);
      d.Ybuf32 = (float*)carve(4 * c->n_y);
    }
    // the scratch keeps whatever the last call on this GPU left: the padding
    // rows of the H slots, which no kernel writes, must read zero
    hipLaunchKernelGGL(k_zero_u64, dim3(1024), dim3(256), 0, c->stream, (unsigned long long*)hbase,
                       (int64_t)(al(hbytes) / 8));
    lrx::TripleLaunch tl = c->tl;
    tl.devs.s[0] = d;
    {
      std::lock_guard<std::mutex> lk(g_plan_mu);
      for (int mt = 0; mt <= lrx::kMaxAlphaTiles; ++mt) tl.mode[mt] = g_tuned[prec][mt] >= 0 ? g_tuned[prec][mt] : 1;
    }
    const lrx::Opts o = make_opts(opts);
    lrx::launch_screen(d, o, c->stream, nullptr);
    lrx::launch_contract(d, tl, prec, c->stream, c->side.data(), c->fork.data(), nullptr, nullptr);
    HIPCHK(hipGetLastError());
    const int N = c->N;
    HIPCHK(hipMemcpyAsync(c->h_out, d.out, sizeof(double) * (1 + 3 * N + 9), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    c->timed = false;
    c->evaluated = true;
    if (E) *E = c->h_out[0];
    if (F) std::memcpy(F, c->h_out + 1, sizeof(double) * 3 * N);
    if (sigma) std::memcpy(sigma, c->h_out + 1 + 3 * N, sizeof(double) * 9);
  });
}

int lrx_hamiltonian(lrx_ctx* c, const lrx_options* opts, double* E, double* Hx, int32_t hx_on_device) {
  return guarded(c, [&] {
    require(!c->bvk, "lrx_hamiltonian: not available with k-point sampling");
    require(c->have_tensors, "evaluation before lrx_set_tensors");
    for (int A = 0; A < c->N; ++A)
      require(c->cp.row[A + 1] - c->cp.row[A] <= lrx::kHxMaxCPartners,
              "lrx_hamiltonian: atom " + std::to_string(A) + " has more than " +
                  std::to_string(lrx::kHxMaxCPartners) + " C partners");
    prepare(c, opts);
    require(opts->precision == LRX_FP64, "the Hamiltonian is computed in FP64 only");
    Dev& d = c->dev;
    const int64_t nt = c->ao[c->N];
    if (!c->have_hx) {
      int kmax = 1;
      for (size_t i = 0; i < c->cp.pA.size(); ++i) kmax = std::max(kmax, c->nao[c->cp.pA[i]] * c->nao[c->cp.pB[i]]);
      c->hx.kmax = kmax;
      c->hx.nmax = *std::max_element(c->nao.begin(), c->nao.end());
      c->hx.Hbar = c->dalloc<double>(c->n_h);
      c->hx.G12 = c->dalloc<double>(nt * nt);
      c->hx.G3 = c->dalloc<double>(nt * nt);
      c->hx.Hx = c->dalloc<double>(nt * nt);
      c->hx.Etile = c->dalloc<double>(lrx::hx_tiles(nt));
      c->hx.E = c->dalloc<double>(1);
      {
        // the D blocks (G,X) that G3 can reach: X of an H slot (B,X) of a C
        // partner B of G (slots are stored by B), in (G, X-first-seen) order,
        // split by the 16-wide tile count of max(nG, nX)
        const int N = c->N;
        require((int64_t)N * N < ((int64_t)1 << 31), "lrx_hamiltonian: more than 46340 atoms");
        const int nSlot = (int)c->slotB.size();
        std::vector<int> srow(N + 1, 0);
        for (int s = 0; s < nSlot; ++s) srow[c->slotB[s] + 1]++;
        for (int B = 0; B < N; ++B) srow[B + 1] += srow[B];
        std::vector<int> blk[2];
        std::vector<int> seen(N, -1);
        for (int G = 0; G < N; ++G)
          for (int i = c->cp.row[G]; i < c->cp.row[G + 1]; ++i) {
            const int B = c->cp.pB[i];
            for (int s = srow[B]; s < srow[B + 1]; ++s) {
              const int X = c->slotX[s];
              if (seen[X] == G) continue;
              seen[X] = G;
              blk[std::max(c->nao[G], c->nao[X]) > 16].push_back(G * N + X);
            }
          }
        for (int k = 0; k < 2; ++k) {
          require(blk[k].size() < ((size_t)1 << 31), "lrx_hamiltonian: too many D blocks");
          c->hx.n3[k] = (int)blk[k].size();
          c->hx.g3blk[k] = c->upload(blk[k]);
        }
      }
      c->have_hx = true;
    }
    const lrx::Opts o = make_opts(opts);
    const bool timing = opts->timing != 0;
    lrx::HxBufs b = c->hx;
    if (hx_on_device && Hx) b.Hx = Hx;   // written straight into the caller's device buffer
    if (timing) HIPCHK(hipEventRecord(c->ev[0], c->stream));
    lrx::launch_screen(d, o, c->stream, nullptr, true);
    if (timing) HIPCHK(hipEventRecord(c->ev[1], c->stream));
    lrx::launch_hbuild(d, lrx::kP64, c->stream);
    if (timing) HIPCHK(hipEventRecord(c->ev[2], c->stream));
    lrx::launch_hx(d, b, c->stream, timing ? c->ev.data() + 3 : nullptr);
    HIPCHK(hipGetLastError());
    double e = 0;
    HIPCHK(hipMemcpyAsync(&e, b.E, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (Hx && !hx_on_device)
      HIPCHK(hipMemcpyAsync(Hx, b.Hx, sizeof(double) * nt * nt, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    if (timing)
      for (int i = 0; i < 5; ++i) HIPCHK(hipEventElapsedTime(&c->hx_ms[i], c->ev[i], c->ev[i + 1]));
    c->hx_timed = timing;
    c->hx_done = true;
    c->per_tensor = (opts->flags & LRX_SCREEN_PER_TENSOR) != 0;
    if (E) *E = e;
  });
}

int lrx_hamiltonian_info(lrx_ctx* c, float* ms, double* flop) {
  return guarded(c, [&] {
    require(c->hx_done, "no Hamiltonian evaluated yet");
    if (ms) {
      require(c->hx_timed, "the last Hamiltonian call was not timed");
      for (int i = 0; i < 5; ++i) ms[i] = c->hx_ms[i];
    }
    if (!flop) return;
    const Dev& d = c->dev;
    const int N = c->N;
    std::vector<uint8_t> aC(d.nCp), aV(d.nVp), need(d.nSlot), kD((size_t)N * N);
    if (d.nCp) HIPCHK(hipMemcpyAsync(aC.data(), d.aliveC, d.nCp, hipMemcpyDeviceToHost, c->stream));
    if (d.nVp) HIPCHK(hipMemcpyAsync(aV.data(), d.aliveV, d.nVp, hipMemcpyDeviceToHost, c->stream));
    if (d.nSlot) HIPCHK(hipMemcpyAsync(need.data(), d.need, d.nSlot, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipMemcpyAsync(kD.data(), d.keepD, (size_t)N * N, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    const auto& na = c->nao;
    const auto& nb = c->nabf;
    const Pairs& cp = c->cp;
    const Pairs& vp = c->vp;
    // per triple with value-list C and V pairs: Q once, and its four
    // contractions (Hbar twice where the D pair is kept, G1 and G2)
    double fs = 0, fg = 0, fh = 0;
    for (int i = 0; i < d.nCp; ++i) {
      if (!(aC[i] & 1)) continue;
      const int A = cp.pA[i], F = cp.pB[i];
      for (int p = vp.row[A]; p < vp.row[A + 1]; ++p) {
        if (!(aV[p] & 1)) continue;
        const int B = vp.pB[p];
        const double k = (double)nb[B] * na[A] * na[F];
        fs += 2.0 * nb[A] * k + 2.0 * k * na[B] * (2 + kD[(size_t)A * N + B] + kD[(size_t)F * N + B]);
      }
    }
    // the H build and its adjoint G3 run over the same (slot, C partner) pairs
    for (int sl = 0; sl < d.nSlot; ++sl) {
      if (!need[sl]) continue;
      const int B = c->slotB[sl], X = c->slotX[sl];
      double depth = 0;
      for (int i = cp.row[B]; i < cp.row[B + 1]; ++i)
        if (aC[i] & 1) depth += na[cp.pB[i]];
      fg += 2.0 * nb[B] * na[B] * na[X] * depth;
    }
    fh = fg;
    flop[0] = fs + fg + fh;
    flop[1] = fs;
    flop[2] = fg;
    flop[3] = fh;
  });
}

int lrx_batch_tuning(const lrx_ctx* c, int32_t* mode, float* ms) {
  if (!c) return LRX_EINVAL;
  for (int mt = 0; mt <= lrx::kMaxAlphaTiles; ++mt) {
    if (mode) mode[mt] = c->tune_mode[mt];
    if (ms) {
      ms[2 * mt] = c->tune_ms[2 * mt];
      ms[2 * mt + 1] = c->tune_ms[2 * mt + 1];
    }
  }
  return lrx::kMaxAlphaTiles + 1;
}

const char* lrx_last_error(const lrx_ctx* c) { return c ? c->err.c_str() : "NULL context"; }

int lrx_pool_trim(int32_t device, uint64_t keep_bytes) {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return LRX_EINVAL;
  if (hipSetDevice(device) != hipSuccess) return LRX_EHIP;
  if (hipDeviceSynchronize() != hipSuccess) return LRX_EHIP;
  (void)lrx::dev_trim(device, (size_t)keep_bytes);
  return LRX_OK;
}

void lrx_destroy(lrx_ctx* c) {
  if (!c) return;
  drop_plans_of(c);
  (void)hipSetDevice(c->device);
  for (auto& kv : c->tickets) {   // submitted and never waited for
    if (kv.second.done) (void)hipEventSynchronize(kv.second.done);
    c->release(kv.second);
  }
  c->tickets.clear();
  c->free_tensors();
  g_pinned.put(c->h_out, c->h_out_bytes);
  if (c->events) {
    for (auto& e : c->ev) (void)hipEventDestroy(e);
    for (auto& e : c->gev) (void)hipEventDestroy(e);
    for (auto& e : c->fork) (void)hipEventDestroy(e);
  }
  for (auto& st : c->side) g_streams.put(c->device, st);
  if (c->own_stream) g_streams.put(c->device, c->stream);
  delete c;
}

}  // extern "C"
