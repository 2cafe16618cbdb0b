// General fused-circuit execution: runs of one- and two-qubit gates applied
// to tiles of the state held in LDS, one HBM pass per run; see
// include/qft_circuit.h.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>
#include <vector>

#include "../../include/qft_circuit.h"
#include "qft_internal.h"

namespace qft {
int set_error(int code, const std::string &msg);
int hip_error(hipError_t e, const char *what);
void clear_error();
}  // namespace qft

using namespace qft;

namespace {

constexpr int kCircThreads = 256;
constexpr int kMaxCircTile = 12;  // 2^12 complex64 / 2^11 complex128 = 32 KiB of LDS

template <typename Real>
struct alignas(2 * sizeof(Real)) c2 {
  Real x, y;
};

enum GateKind : int32_t { kOne = 0, kControlled = 1, kSwap = 2 };

struct GateRec {
  int32_t kind;
  int32_t a, b;    // one-qubit: target a; controlled: control a, target b; swap: a, b
  double u[8];     // row-major 2x2, (re, im) pairs
};

// A gate as a pass applies it: tile-bit positions, matrix in the dtype.
template <typename Real>
struct DevGate {
  int32_t kind, la, lb, pad;
  c2<Real> u[4];
};

struct CircPass {
  int32_t n, T, nfree, ngates;
  uint32_t gpos_w[4];   // global bit of tile position q (packed 4 per word)
  uint32_t free_w[8];   // global bits of the non-tile positions, ascending
  uint32_t ntiles;
  int32_t xcd_remap;
  const void *gates;    // DevGate<Real>[ngates]
};

__device__ __forceinline__ uint32_t insert_zero(uint32_t x, int pos) {
  const uint32_t low = (1u << pos) - 1u;
  return ((x & ~low) << 1) | (x & low);
}

template <typename Real>
__device__ __forceinline__ c2<Real> cmul2(c2<Real> a, c2<Real> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

template <typename Real>
__device__ __forceinline__ c2<Real> cadd2(c2<Real> a, c2<Real> b) {
  return {a.x + b.x, a.y + b.y};
}

// One pass: load the tile into LDS (tile element e = sum of bit q of e at
// global bit gpos[q]), apply the pass's gates in order, store the tile.
template <typename Real>
__global__ void __launch_bounds__(kCircThreads) k_circuit_pass(const CircPass d, c2<Real> *psi) {
  using C = c2<Real>;
  extern __shared__ __align__(16) unsigned char circ_smem[];
  C *lds = reinterpret_cast<C *>(circ_smem);
  uint32_t tile = blockIdx.x;
  if (d.xcd_remap) {
    const uint32_t per = gridDim.x >> 3;
    tile = (blockIdx.x & 7u) * per + (blockIdx.x >> 3);
  }
  uint64_t base = 0;
  for (int b = 0; b < d.nfree; ++b) base |= (uint64_t)((tile >> b) & 1u) << pos_get(d.free_w, b);
  const uint32_t TE = 1u << d.T;
  auto addr = [&](uint32_t e) {
    uint64_t g = base;
    for (int q = 0; q < d.T; ++q) g |= (uint64_t)((e >> q) & 1u) << pos_get(d.gpos_w, q);
    return g;
  };
  for (uint32_t e = threadIdx.x; e < TE; e += kCircThreads) lds[e] = psi[addr(e)];
  __syncthreads();
  const DevGate<Real> *G = (const DevGate<Real> *)d.gates;
  for (int gi = 0; gi < d.ngates; ++gi) {
    const DevGate<Real> g = G[gi];
    if (g.kind == kOne) {
      for (uint32_t p = threadIdx.x; p < (TE >> 1); p += kCircThreads) {
        const uint32_t e0 = insert_zero(p, g.la), e1 = e0 | (1u << g.la);
        const C a = lds[e0], b = lds[e1];
        lds[e0] = cadd2(cmul2(g.u[0], a), cmul2(g.u[1], b));
        lds[e1] = cadd2(cmul2(g.u[2], a), cmul2(g.u[3], b));
      }
    } else if (g.kind == kControlled) {
      const int lo = g.la < g.lb ? g.la : g.lb, hi = g.la < g.lb ? g.lb : g.la;
      for (uint32_t p = threadIdx.x; p < (TE >> 2); p += kCircThreads) {
        const uint32_t e0 = insert_zero(insert_zero(p, lo), hi) | (1u << g.la);
        const uint32_t e1 = e0 | (1u << g.lb);
        const C a = lds[e0], b = lds[e1];
        lds[e0] = cadd2(cmul2(g.u[0], a), cmul2(g.u[1], b));
        lds[e1] = cadd2(cmul2(g.u[2], a), cmul2(g.u[3], b));
      }
    } else {
      const int lo = g.la < g.lb ? g.la : g.lb, hi = g.la < g.lb ? g.lb : g.la;
      for (uint32_t p = threadIdx.x; p < (TE >> 2); p += kCircThreads) {
        const uint32_t z = insert_zero(insert_zero(p, lo), hi);
        const uint32_t e0 = z | (1u << g.la), e1 = z | (1u << g.lb);
        const C a = lds[e0];
        lds[e0] = lds[e1];
        lds[e1] = a;
      }
    }
    __syncthreads();
  }
  for (uint32_t e = threadIdx.x; e < TE; e += kCircThreads) psi[addr(e)] = lds[e];
}

}  // namespace

struct qft_circuit_s {
  int n = 0;
  bool c128 = false;
  int device = 0;
  std::vector<GateRec> gates;
  // compiled form
  bool compiled = false;
  int tile_qubits = 0;
  std::vector<CircPass> passes;
  std::vector<int> gate_begin;  // first gate of each pass
  void *d_gates = nullptr;
};

namespace {

int check_qubit(const qft_circuit_s *c, int q) { return q >= 0 && q < c->n; }

void drop_compiled(qft_circuit_s *c) {
  if (c->d_gates) hipFree(c->d_gates);
  c->d_gates = nullptr;
  c->passes.clear();
  c->gate_begin.clear();
  c->compiled = false;
}

int add_gate(qft_circuit_s *c, const GateRec &g) {
  try {
    c->gates.push_back(g);
  } catch (const std::bad_alloc &) {
    return set_error(QFT_ERR_NOMEM, "out of host memory");
  }
  if (c->compiled) drop_compiled(c);
  return QFT_OK;
}

std::vector<int> gate_qubits(const GateRec &g) {
  if (g.kind == kOne) return {g.a};
  return {g.a, g.b};
}

template <typename Real>
void pack_gate(const GateRec &g, const std::vector<int> &tpos, DevGate<Real> &o) {
  o.kind = g.kind;
  o.la = tpos[g.a];
  o.lb = g.kind == kOne ? 0 : tpos[g.b];
  o.pad = 0;
  for (int i = 0; i < 4; ++i) o.u[i] = c2<Real>{(Real)g.u[2 * i], (Real)g.u[2 * i + 1]};
}

int compile(qft_circuit_s *c, int tile_qubits, bool upload) {
  drop_compiled(c);
  const int n = c->n;
  const int T = std::min(n, c->c128 ? kMaxCircTile - 1 : kMaxCircTile);
  int B = tile_qubits > 0 ? tile_qubits : 10;
  B = std::max(2, std::min(B, T));
  c->tile_qubits = B;
  // greedy runs of gates whose qubits fit in B
  std::vector<std::pair<int, int>> runs;
  std::vector<std::vector<int>> sets;
  {
    std::vector<int> S;
    int start = 0;
    for (int i = 0; i < (int)c->gates.size(); ++i) {
      std::vector<int> U = S;
      for (int q : gate_qubits(c->gates[i]))
        if (std::find(U.begin(), U.end(), q) == U.end()) U.push_back(q);
      if ((int)U.size() > B) {
        runs.push_back({start, i});
        sets.push_back(S);
        start = i;
        U = gate_qubits(c->gates[i]);
        std::sort(U.begin(), U.end());
        U.erase(std::unique(U.begin(), U.end()), U.end());
      }
      S = U;
    }
    if (!c->gates.empty()) {
      runs.push_back({start, (int)c->gates.size()});
      sets.push_back(S);
    }
  }
  const size_t gsz = c->c128 ? sizeof(DevGate<double>) : sizeof(DevGate<float>);
  std::vector<unsigned char> host(c->gates.size() * gsz);
  for (size_t r = 0; r < runs.size(); ++r) {
    std::vector<int> S = sets[r];
    // tile: the run's qubits plus the lowest other qubits, up to T bits,
    // ordered by global bit so that low tile bits give contiguous runs
    std::vector<int> tile = S;
    for (int q = 0; q < n && (int)tile.size() < T; ++q)
      if (std::find(tile.begin(), tile.end(), q) == tile.end()) tile.push_back(q);
    std::sort(tile.begin(), tile.end());
    std::vector<int> tpos(n, -1);
    CircPass p;
    memset(&p, 0, sizeof(p));
    p.n = n;
    p.T = (int)tile.size();
    for (int q = 0; q < p.T; ++q) {
      pos_set(p.gpos_w, q, (uint32_t)tile[q]);
      tpos[tile[q]] = q;
    }
    int nf = 0;
    for (int b = 0; b < n; ++b)
      if (tpos[b] < 0) pos_set(p.free_w, nf++, (uint32_t)b);
    p.nfree = nf;
    p.ntiles = 1u << nf;
    p.xcd_remap = (p.ntiles >= 8 && p.ntiles % 8 == 0) ? 1 : 0;
    p.ngates = runs[r].second - runs[r].first;
    for (int i = runs[r].first; i < runs[r].second; ++i) {
      unsigned char *dst = host.data() + (size_t)i * gsz;
      if (c->c128) pack_gate<double>(c->gates[i], tpos, *(DevGate<double> *)dst);
      else pack_gate<float>(c->gates[i], tpos, *(DevGate<float> *)dst);
    }
    c->passes.push_back(p);
    c->gate_begin.push_back(runs[r].first);
  }
  if (!upload) return QFT_OK;  // host grouping only (describe)
  if (!host.empty()) {
    hipError_t e = hipMalloc(&c->d_gates, host.size());
    if (e != hipSuccess) {
      c->d_gates = nullptr;
      return hip_error(e, "circuit gate upload");
    }
    e = hipMemcpy(c->d_gates, host.data(), host.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_error(e, "circuit gate upload");
  }
  for (size_t r = 0; r < c->passes.size(); ++r)
    c->passes[r].gates = (unsigned char *)c->d_gates + (size_t)c->gate_begin[r] * gsz;
  c->compiled = true;
  return QFT_OK;
}

}  // namespace

extern "C" {

qft_circuit_t *qft_circuit_create(int n, int layout) {
  clear_error();
  if (n < 1 || n > QFT_MAX_QUBITS) {
    set_error(QFT_ERR_INVALID, "n out of range");
    return nullptr;
  }
  qft_circuit_s *c = new (std::nothrow) qft_circuit_s();
  if (!c) {
    set_error(QFT_ERR_NOMEM, "out of host memory");
    return nullptr;
  }
  c->n = n;
  c->c128 = (layout & QFT_C128) != 0;
  if (hipGetDevice(&c->device) != hipSuccess) c->device = 0;
  return c;
}

void qft_circuit_destroy(qft_circuit_t *c) {
  if (!c) return;
  drop_compiled(c);
  delete c;
}

int qft_circuit_add_1q(qft_circuit_t *c, int q, const double u[8]) {
  clear_error();
  if (!c || !u) return set_error(QFT_ERR_INVALID, "NULL argument");
  if (!check_qubit(c, q)) return set_error(QFT_ERR_INVALID, "qubit out of range");
  GateRec g;
  g.kind = kOne;
  g.a = q;
  g.b = -1;
  memcpy(g.u, u, sizeof(g.u));
  return add_gate(c, g);
}

int qft_circuit_add_controlled(qft_circuit_t *c, int control, int target, const double u[8]) {
  clear_error();
  if (!c || !u) return set_error(QFT_ERR_INVALID, "NULL argument");
  if (!check_qubit(c, control) || !check_qubit(c, target) || control == target)
    return set_error(QFT_ERR_INVALID, "bad control / target qubits");
  GateRec g;
  g.kind = kControlled;
  g.a = control;
  g.b = target;
  memcpy(g.u, u, sizeof(g.u));
  return add_gate(c, g);
}

int qft_circuit_add_swap(qft_circuit_t *c, int a, int b) {
  clear_error();
  if (!c) return set_error(QFT_ERR_INVALID, "NULL argument");
  if (!check_qubit(c, a) || !check_qubit(c, b) || a == b)
    return set_error(QFT_ERR_INVALID, "bad swap qubits");
  GateRec g;
  memset(&g, 0, sizeof(g));
  g.kind = kSwap;
  g.a = a;
  g.b = b;
  return add_gate(c, g);
}

int qft_circuit_compile(qft_circuit_t *c, int tile_qubits) {
  clear_error();
  if (!c) return set_error(QFT_ERR_INVALID, "NULL circuit");
  if (tile_qubits < 0) return set_error(QFT_ERR_INVALID, "tile_qubits < 0");
  return compile(c, tile_qubits, true);
}

int qft_circuit_describe(qft_circuit_t *c, int tile_qubits, int *gate_begin, int *tile_bits,
                         int max_passes) {
  clear_error();
  if (!c) return set_error(QFT_ERR_INVALID, "NULL circuit");
  if (tile_qubits < 0) return set_error(QFT_ERR_INVALID, "tile_qubits < 0");
  int rc = compile(c, tile_qubits, false);
  if (rc != QFT_OK) return rc;
  const int np = (int)c->passes.size();
  for (int i = 0; i < np && i < max_passes; ++i) {
    if (gate_begin) gate_begin[i] = c->gate_begin[i];
    if (tile_bits) tile_bits[i] = c->passes[i].T;
  }
  drop_compiled(c);
  return np;
}

int qft_circuit_info(const qft_circuit_t *c, int *gates, int *passes) {
  clear_error();
  if (!c) return set_error(QFT_ERR_INVALID, "NULL circuit");
  if (gates) *gates = (int)c->gates.size();
  if (passes) *passes = c->compiled ? (int)c->passes.size() : -1;
  return QFT_OK;
}

int qft_circuit_execute(qft_circuit_t *c, void *dev_ptr, qft_stream_t stream) {
  clear_error();
  if (!c) return set_error(QFT_ERR_INVALID, "NULL circuit");
  if (!dev_ptr) return set_error(QFT_ERR_POINTER, "data pointer is NULL");
  if ((uintptr_t)dev_ptr % (c->c128 ? 16 : 8))
    return set_error(QFT_ERR_POINTER, "data pointer is not aligned to the element size");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev != c->device)
    return set_error(QFT_ERR_INVALID, "the current device is not the circuit's device");
  if (!c->compiled) {
    int rc = compile(c, c->tile_qubits, true);
    if (rc != QFT_OK) return rc;
  }
  hipStream_t s = (hipStream_t)stream;
  for (const CircPass &p : c->passes) {
    const size_t lds = ((size_t)1 << p.T) * (c->c128 ? 16 : 8);
    if (c->c128)
      hipLaunchKernelGGL(k_circuit_pass<double>, dim3(p.ntiles), dim3(kCircThreads), lds, s, p,
                         (c2<double> *)dev_ptr);
    else
      hipLaunchKernelGGL(k_circuit_pass<float>, dim3(p.ntiles), dim3(kCircThreads), lds, s, p,
                         (c2<float> *)dev_ptr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_error(e, "circuit pass launch");
  }
  return QFT_OK;
}

}  // extern "C"
