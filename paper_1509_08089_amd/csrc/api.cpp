// C ABI: graphs, table build, plain estimation.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"

namespace moss {

moss_status status_of(hipError_t e) {
  if (e == hipSuccess) return MOSS_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return MOSS_E_NOMEM;
  return MOSS_E_DEVICE;
}

DeviceScope::DeviceScope(int device) {
  if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
  ok_ = hipSetDevice(device) == hipSuccess;
}

DeviceScope::~DeviceScope() {
  if (prev_ >= 0) (void)hipSetDevice(prev_);
}

GraphClaim::GraphClaim(moss_graph* g) : g_(g) {
  int expected = 0;
  ok_ = g && g->busy.compare_exchange_strong(expected, 1);
}

GraphClaim::~GraphClaim() {
  if (ok_) g_->busy.store(0);
}

namespace {
std::mutex g_dev_mu;
std::vector<int> g_dev_ready;  // per device: 0 not set up, 1 ready
std::vector<int> g_dev_cus;
}  // namespace

moss_status ensure_device(int device) {
  std::lock_guard<std::mutex> lk(g_dev_mu);
  if (device < 0) return MOSS_E_DEVICE;
  if ((int)g_dev_ready.size() <= device) {
    g_dev_ready.resize(device + 1, 0);
    g_dev_cus.resize(device + 1, 0);
  }
  if (g_dev_ready[device]) return MOSS_OK;
  DeviceScope scope(device);
  if (!scope.ok()) return MOSS_E_DEVICE;
  uint8_t l4[8], lt[64], lp[64];
  class_luts(l4, lt, lp);
  hipError_t e = upload_class_luts(l4, lt, lp);
  if (e != hipSuccess) return status_of(e);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
    return MOSS_E_DEVICE;
  hipMemPool_t pool = nullptr;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess && pool) {
    uint64_t keep = ~0ull;  // keep freed blocks for reuse instead of returning them at each sync
    (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
  }
  g_dev_cus[device] = cus;
  g_dev_ready[device] = 1;
  return MOSS_OK;
}

int device_cus(int device) {
  std::lock_guard<std::mutex> lk(g_dev_mu);
  return device >= 0 && device < (int)g_dev_cus.size() && g_dev_cus[device] > 0 ? g_dev_cus[device] : 256;
}

SamplerView sampler_view(const moss_graph* g, int sampler) {
  const int s = sampler_slot(sampler);
  SamplerView v{};
  v.rp = g->rp;
  v.col = g->col;
  v.acc_node = g->acc_node[s];
  v.guide = g->guide[s];
  v.acc_sigma = g->acc_sigma;
  v.acc_tau = g->acc_tau;
  v.rec = g->rec;
  v.sig_guide = g->sig_guide;
  v.tau_guide = g->tau_guide;
  v.edge_slots = g->edge_slots;
  v.edge_bits = g->edge_bits;
  v.total = g->total[s];
  v.n = g->n;
  v.gbits = g->gbits;
  return v;
}

void plain_launch_shape(int device, int sampler, uint64_t nsamples, int* grid, int* block) {
  const Tuning t = current_tuning();
  int b = t.threads_per_block ? (int)t.threads_per_block : 256;
  int per_cu = t.blocks_per_cu ? (int)t.blocks_per_cu : 0;
  if (per_cu == 0) {
    per_cu = sample_kernel_blocks_per_cu(sampler, b);
    per_cu = std::max(1, std::min(per_cu, 8));
  }
  const uint64_t want = (nsamples + (uint64_t)b - 1) / (uint64_t)b;
  const uint64_t cap = (uint64_t)device_cus(device) * (uint64_t)per_cu;
  *grid = (int)std::max<uint64_t>(1, std::min(want, cap));
  *block = b;
}

}  // namespace moss

using namespace moss;

namespace {

// Device memory is stream-ordered (hipMallocAsync on the graph's stream from the
// device's default pool, which keeps freed blocks for reuse), so building and
// dropping tables costs no device-wide synchronisation.
template <typename T>
moss_status dev_alloc(hipStream_t s, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMallocAsync((void**)p, count * sizeof(T), s);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return MOSS_E_NOMEM;
  }
  return MOSS_OK;
}

template <typename T>
void dev_free(hipStream_t s, T*& p) {
  if (p) (void)hipFreeAsync((void*)p, s);
  p = nullptr;
}

// Small pinned host buffers for results and flags, reused across graphs.
std::mutex g_pin_mu;
std::vector<uint64_t*> g_pin_free;
constexpr size_t kPinWords = 64;

uint64_t* pinned_chunk() {
  std::lock_guard<std::mutex> lk(g_pin_mu);
  if (g_pin_free.empty()) {
    uint64_t* slab = nullptr;
    if (hipHostMalloc((void**)&slab, 64 * kPinWords * sizeof(uint64_t), hipHostMallocDefault) != hipSuccess)
      return nullptr;
    for (int i = 0; i < 64; ++i) g_pin_free.push_back(slab + i * kPinWords);
  }
  uint64_t* p = g_pin_free.back();
  g_pin_free.pop_back();
  return p;
}

void pinned_release(uint64_t* p) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_free.push_back(p);
}

void free_tables(moss_graph* g, uint32_t mask) {
  if (mask & MOSS_TABLES_K4) {
    dev_free(g->stream, g->acc_node[0]);
    dev_free(g->stream, g->guide[0]);
    g->total[0] = 0;
  }
  if (mask & MOSS_TABLES_K5) {
    dev_free(g->stream, g->acc_node[1]);
    dev_free(g->stream, g->acc_node[2]);
    dev_free(g->stream, g->guide[1]);
    dev_free(g->stream, g->guide[2]);
    dev_free(g->stream, g->acc_tau);
    dev_free(g->stream, g->tau_guide);
    g->total[1] = g->total[2] = 0;
  }
  g->built &= ~mask;
  if (!(g->built & (MOSS_TABLES_K4 | MOSS_TABLES_K5))) {
    dev_free(g->stream, g->acc_sigma);
    dev_free(g->stream, g->sig_guide);
    dev_free(g->stream, g->edge_slots);
    g->sigma_ready = false;
  }
  g->table_bytes = moss::table_bytes_needed(g, 0);
}

void destroy_graph(moss_graph* g) {
  if (!g) return;
  DeviceScope scope(g->device);
  (void)hipStreamSynchronize(g->stream);
  free_tables(g, MOSS_TABLES_K4 | MOSS_TABLES_K5);
  dev_free(g->stream, g->owned_rp);
  dev_free(g->stream, g->owned_col);
  dev_free(g->stream, g->items);
  dev_free(g->stream, g->item_sum);
  dev_free(g->stream, g->scan_tmp);
  dev_free(g->stream, g->partials);
  dev_free(g->stream, g->rec);
  dev_free(g->stream, g->d_hits);
  dev_free(g->stream, g->d_err);
  dev_free(g->stream, g->d_lambda);
  dev_free(g->stream, g->d_meta);
  pinned_release(g->h_stage);
  g->h_stage = nullptr;
  if (g->ev0) (void)hipEventDestroy(g->ev0);
  if (g->ev1) (void)hipEventDestroy(g->ev1);
  delete g;
}

int validate_error_status(uint32_t bits) {
  if (bits & kErrArg) return MOSS_E_ARG;
  if (bits & kErrSelfLoop) return MOSS_E_SELF_LOOP;
  if (bits & kErrDuplicate) return MOSS_E_DUPLICATE;
  if (bits & kErrUnsorted) return MOSS_E_UNSORTED;
  if (bits & kErrAsymmetric) return MOSS_E_ASYMMETRIC;
  if (bits & kErrOverflow) return MOSS_E_OVERFLOW;
  return MOSS_OK;
}

// Scratch, events and the CSR checks shared by both creation paths.
moss_status finish_create(moss_graph* g) {
  moss_status st;
  if ((st = dev_alloc(g->stream, &g->d_hits, 2 * 22)) != MOSS_OK) return st;
  if ((st = dev_alloc(g->stream, &g->d_err, 4)) != MOSS_OK) return st;
  if ((st = dev_alloc(g->stream, &g->d_lambda, 2)) != MOSS_OK) return st;
  if ((st = dev_alloc(g->stream, &g->d_meta, 2)) != MOSS_OK) return st;
  if (!(g->h_stage = pinned_chunk())) return MOSS_E_NOMEM;
  if (hipEventCreate(&g->ev0) != hipSuccess || hipEventCreate(&g->ev1) != hipSuccess) return MOSS_E_DEVICE;
  hipStream_t s = g->stream;
  hipError_t e = launch_fill_u32(g->d_err, 0, 4, s);
  if (e == hipSuccess) e = launch_check_rowptr(g->n, g->nnz, g->rp, g->d_err, s);
  if (e == hipSuccess) e = hipMemcpyAsync(g->h_stage, g->d_err, 2 * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return status_of(e);
  uint32_t bits = ((uint32_t*)g->h_stage)[0];
  g->max_degree = (int32_t)((uint32_t*)g->h_stage)[1];
  if (bits) return (moss_status)validate_error_status(bits);
  // work items: every row cut into pieces of at most 256 entries
  const int64_t items_ub = (int64_t)g->n + g->nnz / 256 + 1;
  const int64_t tmp_elems = std::max(scan_tmp_elems(g->n), scan_tmp_elems(items_ub));
  uint64_t* item_end = nullptr;
  if ((st = dev_alloc(g->stream, &g->items, (size_t)items_ub)) != MOSS_OK) return st;
  if ((st = dev_alloc(g->stream, &g->item_sum, (size_t)items_ub)) != MOSS_OK) return st;
  if ((st = dev_alloc(g->stream, &g->scan_tmp, (size_t)tmp_elems)) != MOSS_OK) return st;
  if ((st = dev_alloc(g->stream, &g->partials, 2 * (size_t)node_weight_blocks(g->n))) != MOSS_OK) return st;
  if ((st = dev_alloc(g->stream, &g->rec, (size_t)g->n)) != MOSS_OK) return st;
  if ((st = dev_alloc(g->stream, &item_end, (size_t)g->n)) != MOSS_OK) return st;
  e = launch_items(g->n, g->rp, item_end, g->items, g->scan_tmp, g->d_err, s);
  if (e == hipSuccess) e = launch_fill_u64(g->d_meta, 0, 2, s);
  if (e == hipSuccess && g->n > 0)
    e = hipMemcpyAsync(g->d_meta, item_end + (g->n - 1), sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
  // row-guide layout (depends on degrees only), then the records' row start, degree, offset
  if (e == hipSuccess) e = launch_row_guide_sizes(g->n, g->rp, item_end, s);
  if (e == hipSuccess) e = launch_scan_inplace(item_end, g->n, g->scan_tmp, g->d_err, kErrArg, s);
  if (e == hipSuccess) e = launch_records(g->n, g->rp, nullptr, item_end, g->rec, s);
  if (e == hipSuccess && g->n > 0)
    e = hipMemcpyAsync(g->d_meta + 1, item_end + (g->n - 1), sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess)
    e = launch_check_items(items_ub, g->d_meta, g->items, g->n, g->rp, g->col, !(g->flags & MOSS_TRUST_CSR),
                           g->d_err, s);
  if (e == hipSuccess) e = hipMemcpyAsync(g->h_stage + 1, g->d_meta, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipMemcpyAsync(g->h_stage, g->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  dev_free(g->stream, item_end);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return status_of(e);
  g->n_items = (int64_t)g->h_stage[1];
  g->row_guide_len = (int64_t)g->h_stage[2];
  if (g->n_items > items_ub) return MOSS_E_ARG;
  bits = ((uint32_t*)g->h_stage)[0];
  return (moss_status)validate_error_status(bits);
}

moss_status create_common(int32_t n, int64_t nnz, uint32_t flags, void* hip_stream, moss_graph** out,
                          moss_graph** made) {
  *made = nullptr;
  if (!out || n < 0 || nnz < 0 || nnz >= (int64_t)1 << 31 || (n == 0 && nnz != 0)) return MOSS_E_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return MOSS_E_DEVICE;
  moss_status st = ensure_device(dev);
  if (st != MOSS_OK) return st;
  moss_graph* g = new (std::nothrow) moss_graph();
  if (!g) return MOSS_E_NOMEM;
  g->device = dev;
  g->stream = (hipStream_t)hip_stream;
  g->n = n;
  g->nnz = nnz;
  g->flags = flags;
  int bits = 1;
  while (bits < 30 && (1ll << bits) < 2ll * (int64_t)std::max(n, 1)) ++bits;
  g->gbits = std::min(bits, 23);
  *made = g;
  return MOSS_OK;
}

}  // namespace

extern "C" {

const char* moss_status_string(moss_status s) {
  switch (s) {
    case MOSS_OK: return "ok";
    case MOSS_E_ARG: return "invalid argument or malformed CSR";
    case MOSS_E_UNSORTED: return "CSR row not strictly ascending";
    case MOSS_E_SELF_LOOP: return "self-loop in CSR";
    case MOSS_E_DUPLICATE: return "duplicate neighbour in CSR";
    case MOSS_E_ASYMMETRIC: return "CSR not symmetric";
    case MOSS_E_OVERFLOW: return "integer overflow in sampling tables";
    case MOSS_E_NOMEM: return "out of memory";
    case MOSS_E_DEVICE: return "HIP device error";
    case MOSS_E_NOT_BUILT: return "tables not built";
    case MOSS_E_BUSY: return "graph busy";
    case MOSS_E_TIMEOUT: return "timed out";
    case MOSS_E_CANCELLED: return "cancelled";
    case MOSS_E_ADMISSION: return "request can never be admitted";
  }
  return "unknown status";
}

moss_status moss_graph_create(int32_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col, uint32_t flags,
                              void* hip_stream, moss_graph** out) {
  if (!row_ptr || (nnz > 0 && !col)) return MOSS_E_ARG;
  moss_graph* g = nullptr;
  moss_status st = create_common(n, nnz, flags, hip_stream, out, &g);
  if (st != MOSS_OK) return st;
  DeviceScope scope(g->device);
  st = dev_alloc(g->stream, &g->owned_rp, (size_t)n + 1);
  if (st == MOSS_OK) st = dev_alloc(g->stream, &g->owned_col, (size_t)nnz);
  if (st == MOSS_OK) {
    hipError_t e = hipMemcpyAsync(g->owned_rp, row_ptr, ((size_t)n + 1) * sizeof(int32_t), hipMemcpyHostToDevice,
                                  g->stream);
    if (e == hipSuccess && nnz > 0)
      e = hipMemcpyAsync(g->owned_col, col, (size_t)nnz * sizeof(int32_t), hipMemcpyHostToDevice, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    st = status_of(e);
  }
  if (st == MOSS_OK) {
    g->rp = g->owned_rp;
    g->col = g->owned_col;
    g->csr_bytes = ((uint64_t)n + 1 + (uint64_t)nnz) * sizeof(int32_t);
    st = finish_create(g);
  }
  if (st != MOSS_OK) {
    destroy_graph(g);
    return st;
  }
  *out = g;
  return MOSS_OK;
}

moss_status moss_graph_create_device(int32_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col,
                                     uint32_t flags, void* hip_stream, moss_graph** out) {
  if (!d_row_ptr || (nnz > 0 && !d_col)) return MOSS_E_ARG;
  moss_graph* g = nullptr;
  moss_status st = create_common(n, nnz, flags, hip_stream, out, &g);
  if (st != MOSS_OK) return st;
  DeviceScope scope(g->device);
  g->rp = d_row_ptr;
  g->col = d_col;
  st = finish_create(g);
  if (st != MOSS_OK) {
    destroy_graph(g);
    return st;
  }
  *out = g;
  return MOSS_OK;
}

moss_status moss_graph_destroy(moss_graph* g) {
  if (!g) return MOSS_E_ARG;
  if (g->busy.load() != 0) return MOSS_E_BUSY;
  destroy_graph(g);
  return MOSS_OK;
}

moss_status moss_build_tables(moss_graph* g, uint32_t k_mask) {
  GraphClaim claim(g);
  if (!g) return MOSS_E_ARG;
  if (!claim.ok()) return MOSS_E_BUSY;
  return build_tables(g, k_mask);
}

moss_status moss_graph_get_info(const moss_graph* g, moss_graph_info* info) {
  if (!g || !info) return MOSS_E_ARG;
  moss_graph_info r{};
  r.n = g->n;
  r.max_degree = g->max_degree;
  r.nnz = g->nnz;
  r.built_mask = g->built;
  r.gamma = g->total[0];
  r.gamma1 = g->total[1];
  r.gamma2 = g->total[2];
  r.lambda3 = g->lambda3;
  r.lambda4 = g->lambda4;
  r.device_bytes = g->table_bytes + (g->owned_rp ? g->csr_bytes : 0);
  *info = r;
  return MOSS_OK;
}

moss_status moss_table_read(const moss_graph* g, int32_t which, void* host_out, int64_t count) {
  if (!g || !host_out) return MOSS_E_ARG;
  const void* src = nullptr;
  size_t bytes = 0;
  switch (which) {
    case MOSS_TAB_ACC_GAMMA:
    case MOSS_TAB_ACC_GAMMA1:
    case MOSS_TAB_ACC_GAMMA2: {
      if (count != g->n) return MOSS_E_ARG;
      const int s = which - MOSS_TAB_ACC_GAMMA;
      if (!(g->built & (s == 0 ? MOSS_TABLES_K4 : MOSS_TABLES_K5))) return MOSS_E_NOT_BUILT;
      src = g->acc_node[s];
      bytes = (size_t)g->n * sizeof(uint64_t);
      break;
    }
    case MOSS_TAB_ACC_SIGMA:
      if (count != g->nnz) return MOSS_E_ARG;
      if (!g->built) return MOSS_E_NOT_BUILT;
      src = g->acc_sigma;
      bytes = (size_t)g->nnz * sizeof(uint32_t);
      break;
    case MOSS_TAB_ACC_TAU:
      if (count != g->nnz) return MOSS_E_ARG;
      if (!(g->built & MOSS_TABLES_K5)) return MOSS_E_NOT_BUILT;
      src = g->acc_tau;
      bytes = (size_t)g->nnz * sizeof(uint64_t);
      break;
    default:
      return MOSS_E_ARG;
  }
  if (bytes == 0) return MOSS_OK;
  DeviceScope scope(g->device);
  hipError_t e = hipMemcpyAsync(host_out, src, bytes, hipMemcpyDeviceToHost, g->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
  return status_of(e);
}

}  // extern "C"

moss_status moss::build_tables(moss_graph* g, uint32_t k_mask) {
  if (k_mask & ~(MOSS_TABLES_K4 | MOSS_TABLES_K5)) return MOSS_E_ARG;
  const uint32_t need = k_mask & ~g->built;
  if (!need) return MOSS_OK;
  DeviceScope scope(g->device);
  if (!scope.ok()) return MOSS_E_DEVICE;
  const bool want4 = need & MOSS_TABLES_K4, want5 = need & MOSS_TABLES_K5;
  const size_t n = (size_t)g->n, nnz = (size_t)g->nnz, G = ((size_t)1 << g->gbits) + 1;
  moss_status st = MOSS_OK;
  uint64_t bytes = 0;
  if (!g->acc_sigma) {
    st = dev_alloc(g->stream, &g->acc_sigma, nnz);
    if (st == MOSS_OK) st = dev_alloc(g->stream, &g->sig_guide, (size_t)g->row_guide_len);
    g->edge_bits = edge_hash_bits(g->nnz / 2);
    if (st == MOSS_OK) st = dev_alloc(g->stream, &g->edge_slots, (size_t)1 << g->edge_bits);
    bytes += nnz * 4;
  }
  if (st == MOSS_OK && want4) {
    st = dev_alloc(g->stream, &g->acc_node[0], n);
    if (st == MOSS_OK) st = dev_alloc(g->stream, &g->guide[0], G);
    bytes += n * 8 + G * 4;
  }
  if (st == MOSS_OK && want5) {
    st = dev_alloc(g->stream, &g->acc_tau, nnz);
    if (st == MOSS_OK) st = dev_alloc(g->stream, &g->tau_guide, (size_t)g->row_guide_len);
    if (st == MOSS_OK) st = dev_alloc(g->stream, &g->acc_node[1], n);
    if (st == MOSS_OK) st = dev_alloc(g->stream, &g->acc_node[2], n);
    if (st == MOSS_OK) st = dev_alloc(g->stream, &g->guide[1], G);
    if (st == MOSS_OK) st = dev_alloc(g->stream, &g->guide[2], G);
    bytes += nnz * 8 + 2 * n * 8 + 2 * G * 4;
  }
  if (st != MOSS_OK) {
    free_tables(g, need);
    return st;
  }
  hipStream_t s = g->stream;
  hipError_t e = launch_fill_u32(g->d_err, 0, 4, s);
  if (e == hipSuccess) e = launch_fill_u64((uint64_t*)g->d_lambda, 0, 2, s);
  if (e == hipSuccess && !g->sigma_ready) {
    e = launch_row_prefix(false, g->n_items, g->items, g->rp, g->col, g->acc_sigma, nullptr, g->item_sum, g->scan_tmp,
                          g->d_err, s);
    if (e == hipSuccess) e = launch_records(g->n, g->rp, g->acc_sigma, nullptr, g->rec, s);
    if (e == hipSuccess)
      e = launch_row_guides(false, g->n_items, g->items, g->rp, g->rec, g->acc_sigma, nullptr, g->sig_guide, s);
    if (e == hipSuccess)
      e = launch_edge_hash(g->n_items, g->items, g->rp, g->col, g->edge_slots, g->edge_bits, g->d_err, s);
  }
  if (e == hipSuccess && want5) {
    e = launch_row_prefix(true, g->n_items, g->items, g->rp, g->col, g->acc_sigma, g->acc_tau, g->item_sum,
                          g->scan_tmp, g->d_err, s);
    if (e == hipSuccess)
      e = launch_row_guides(true, g->n_items, g->items, g->rp, g->rec, nullptr, g->acc_tau, g->tau_guide, s);
  }
  if (e == hipSuccess)
    e = launch_node_weights(g->n, g->rp, g->acc_sigma, want5 ? g->acc_tau : nullptr, want4 ? g->acc_node[0] : nullptr,
                            want5 ? g->acc_node[1] : nullptr, want5 ? g->acc_node[2] : nullptr, g->partials,
                            g->d_lambda, g->d_err, s);
  for (int slot = 0; slot < 3 && e == hipSuccess; ++slot) {
    const bool want = slot == 0 ? want4 : want5;
    if (want)
      e = launch_scan_inplace(g->acc_node[slot], (int64_t)n, g->scan_tmp, g->d_err,
                              slot == 0 ? kErrOverflowK4 : kErrOverflowK5, s);
  }
  for (int slot = 0; slot < 3 && e == hipSuccess; ++slot) {
    const bool want = slot == 0 ? want4 : want5;
    if (want) e = launch_guide(g->acc_node[slot], g->n, g->gbits, g->guide[slot], s);
  }
  // stage: [0] error bits, [1..3] totals, [4..5] Lambdas
  uint64_t* h = g->h_stage;
  if (e == hipSuccess) e = hipMemcpyAsync(h, g->d_err, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
  for (int slot = 0; slot < 3 && e == hipSuccess; ++slot) {
    const bool want = slot == 0 ? want4 : want5;
    h[1 + slot] = 0;
    if (want && n > 0)
      e = hipMemcpyAsync(h + 1 + slot, g->acc_node[slot] + (n - 1), sizeof(uint64_t), hipMemcpyDeviceToHost, s);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(h + 4, g->d_lambda, 2 * sizeof(uint64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    free_tables(g, need);
    return status_of(e);
  }
  const uint32_t bits = (uint32_t)(h[0] & 0xFFFFFFFFu);
  if ((bits & kErrOverflow) || (want4 && (bits & kErrOverflowK4)) || (want5 && (bits & kErrOverflowK5))) {
    free_tables(g, need);
    return MOSS_E_OVERFLOW;
  }
  g->sigma_ready = true;
  for (int slot = 0; slot < 3; ++slot) {
    const bool want = slot == 0 ? want4 : want5;
    if (want) g->total[slot] = h[1 + slot];
  }
  g->lambda3 = h[4];
  g->lambda4 = h[5];
  g->built |= need;
  g->table_bytes = table_bytes_needed(g, 0);
  (void)bytes;
  return MOSS_OK;
}

void moss::free_graph_tables(moss_graph* g, uint32_t mask) {
  DeviceScope scope(g->device);
  (void)hipStreamSynchronize(g->stream);
  free_tables(g, mask & (MOSS_TABLES_K4 | MOSS_TABLES_K5));
}

// With mask = 0: the bytes held now.  Otherwise the bytes that building `mask` adds.
uint64_t moss::table_bytes_needed(const moss_graph* g, uint32_t mask) {
  const uint64_t n = (uint64_t)g->n, nnz = (uint64_t)g->nnz, G = (1ull << g->gbits) + 1;
  const uint64_t rg = (uint64_t)g->row_guide_len * 4;
  const uint64_t hash = 8ull << edge_hash_bits(g->nnz / 2);
  const uint64_t k4 = n * 8 + G * 4, k5 = nnz * 8 + 2 * n * 8 + 2 * G * 4 + rg, sig = nnz * 4 + rg + hash;
  if (mask == 0) {
    uint64_t b = 0;
    if (g->built) b += sig;
    if (g->built & MOSS_TABLES_K4) b += k4;
    if (g->built & MOSS_TABLES_K5) b += k5;
    return b;
  }
  const uint32_t need = mask & ~g->built;
  uint64_t b = 0;
  if (need && !g->built) b += sig;
  if (need & MOSS_TABLES_K4) b += k4;
  if (need & MOSS_TABLES_K5) b += k5;
  return b;
}

namespace {

// Runs the samplers of one estimate on the graph's stream; hits are copied to `hits`.
moss_status run_samplers(moss_graph* g, const int* samplers, const uint64_t* k0, const uint64_t* k1, int count,
                         uint64_t seed, uint8_t* class_out, uint64_t hits[][22], double* device_ms) {
  hipStream_t s = g->stream;
  hipError_t e = launch_fill_u64((uint64_t*)g->d_hits, 0, 2 * 22, s);
  if (e == hipSuccess) e = hipEventRecord(g->ev0, s);
  for (int i = 0; i < count && e == hipSuccess; ++i) {
    const int slot = sampler_slot(samplers[i]);
    if (g->total[slot] == 0 || k1[i] <= k0[i]) continue;
    int grid, block;
    plain_launch_shape(g->device, samplers[i], k1[i] - k0[i], &grid, &block);
    e = launch_sample(samplers[i], sampler_view(g, samplers[i]), seed, k0[i], k1[i], g->d_hits + 22 * i, class_out,
                      grid, block, s);
  }
  if (e == hipSuccess) e = hipEventRecord(g->ev1, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(g->h_stage, g->d_hits, 2 * 22 * sizeof(uint64_t), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return status_of(e);
  for (int i = 0; i < count; ++i) std::memcpy(hits[i], g->h_stage + 22 * i, 22 * sizeof(uint64_t));
  float ms = 0.f;
  if (device_ms) *device_ms = hipEventElapsedTime(&ms, g->ev0, g->ev1) == hipSuccess ? (double)ms : 0.0;
  return MOSS_OK;
}

bool valid_sampler(int s) { return s == kMoss4 || s == kT5 || s == kPath5; }

}  // namespace

extern "C" {

moss_status moss_estimate(moss_graph* g, int32_t k, uint64_t n_samples, uint64_t seed, uint32_t flags,
                          moss_result* out) {
  if (!g || !out || (k != 4 && k != 5) || (flags & ~MOSS_MIX_PAPER)) return MOSS_E_ARG;
  if ((k == 4 && n_samples < 1) || (k == 5 && n_samples < 2)) return MOSS_E_ARG;
  GraphClaim claim(g);
  if (!claim.ok()) return MOSS_E_BUSY;
  DeviceScope scope(g->device);
  if (!scope.ok()) return MOSS_E_DEVICE;
  moss_status st = build_tables(g, k == 4 ? MOSS_TABLES_K4 : MOSS_TABLES_K5);
  if (st != MOSS_OK) return st;
  moss_result r{};
  r.k = k;
  r.flags = flags;
  r.n_samples = n_samples;
  int samplers[2];
  uint64_t k0[2] = {0, 0}, k1[2];
  int count;
  if (k == 4) {
    r.K[0] = n_samples;
    r.gamma[0] = g->total[0];
    r.lambda = g->lambda3;
    samplers[0] = kMoss4;
    k1[0] = n_samples;
    count = 1;
  } else {
    r.K[0] = (n_samples + 1) / 2;
    r.K[1] = n_samples / 2;
    r.gamma[0] = g->total[1];
    r.gamma[1] = g->total[2];
    r.lambda = g->lambda4;
    samplers[0] = kT5;
    samplers[1] = kPath5;
    k1[0] = r.K[0];
    k1[1] = r.K[1];
    count = 2;
  }
  st = run_samplers(g, samplers, k0, k1, count, seed, nullptr, r.hits, &r.device_ms);
  if (st != MOSS_OK) return st;
  st = moss_finals(&r);
  if (st != MOSS_OK) return st;
  *out = r;
  return MOSS_OK;
}

moss_status moss_sample_range(moss_graph* g, int32_t sampler, uint64_t seed, uint64_t k0, uint64_t k1,
                              uint8_t* d_class_out, uint64_t hits[22]) {
  if (!g || !hits || !valid_sampler(sampler) || k1 < k0) return MOSS_E_ARG;
  GraphClaim claim(g);
  if (!claim.ok()) return MOSS_E_BUSY;
  DeviceScope scope(g->device);
  if (!scope.ok()) return MOSS_E_DEVICE;
  moss_status st = build_tables(g, sampler == kMoss4 ? MOSS_TABLES_K4 : MOSS_TABLES_K5);
  if (st != MOSS_OK) return st;
  uint64_t h[2][22];
  const int samplers[1] = {sampler};
  const uint64_t a[1] = {k0}, b[1] = {k1};
  if (d_class_out && g->total[sampler_slot(sampler)] == 0 && k1 > k0) {
    hipError_t e = hipMemsetAsync(d_class_out, 0, (size_t)(k1 - k0), g->stream);
    if (e != hipSuccess) return status_of(e);
  }
  st = run_samplers(g, samplers, a, b, 1, seed, d_class_out, h, nullptr);
  if (st != MOSS_OK) return st;
  std::memcpy(hits, h[0], sizeof(h[0]));
  return MOSS_OK;
}

moss_status moss_sample_nodes(moss_graph* g, int32_t sampler, uint64_t seed, const uint64_t* d_index, int64_t count,
                              int32_t* d_nodes_out, uint8_t* d_class_out) {
  if (!g || !valid_sampler(sampler) || count < 0 || (count > 0 && (!d_index || !d_nodes_out))) return MOSS_E_ARG;
  GraphClaim claim(g);
  if (!claim.ok()) return MOSS_E_BUSY;
  DeviceScope scope(g->device);
  if (!scope.ok()) return MOSS_E_DEVICE;
  moss_status st = build_tables(g, sampler == kMoss4 ? MOSS_TABLES_K4 : MOSS_TABLES_K5);
  if (st != MOSS_OK) return st;
  if (g->total[sampler_slot(sampler)] == 0) return count == 0 ? MOSS_OK : MOSS_E_ARG;  // nothing can be drawn
  hipError_t e = launch_sample_nodes(sampler, sampler_view(g, sampler), seed, d_index, count, d_nodes_out,
                                     d_class_out, g->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
  return status_of(e);
}

}  // extern "C"
