// Grid hierarchy and FP64 operator constants (host side).
//
// The multilevel decomposition of the paper (Sec. 2) on a structured tensor
// grid, read as the P1 finite-element hierarchy:
//   * a side of n nodes coarsens to floor(n/2)+1 nodes (even indices plus the
//     last index); sides of 1 or 2 nodes are not decomposed; all decomposed
//     sides coarsen together, L = the fewest coarsenings that bring one of
//     them to 3 nodes;
//   * per level and dimension: linear interpolation weights of the new nodes,
//     the consistent P1 mass matrix, the restriction (transposed
//     interpolation) and the Thomas factors of the coarse mass matrix;
//   * K_l = prod_d ||T^-1 P^T M||_inf and S = 1 + sum_l (1 + K_l), the constant
//     of the a-priori L-infinity bound used by the plain bin allocation.
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>

#include "internal.hpp"

namespace mg {

namespace {

int dim_levels(int64_t n) {
  if (n <= 2) return -1;
  int k = 0;
  while (n > 3) {
    n = n / 2 + 1;
    ++k;
  }
  return k;
}

void mass_bands(const std::vector<double>& x, std::vector<double>& a, std::vector<double>& b,
                std::vector<double>& c) {
  const size_t n = x.size();
  a.assign(n, 0.0);
  b.assign(n, 0.0);
  c.assign(n, 0.0);
  for (size_t i = 0; i < n; ++i) {
    double hl = i > 0 ? x[i] - x[i - 1] : 0.0;
    double hr = i + 1 < n ? x[i + 1] - x[i] : 0.0;
    b[i] = (hl + hr) / 3.0;
    if (i > 0) a[i] = hl / 6.0;
    if (i + 1 < n) c[i] = hr / 6.0;
  }
}

// Row sums of |T^-1 P^T M|, one column at a time: column k of P^T M has at
// most three nonzeros, and each column is solved with the same Thomas
// factors.  Returns the maximum row sum.
double correction_norm(const DimOps& o) {
  const int nf = o.nf, nc = o.nc;
  std::vector<double> rows(nc, 0.0), col(nc), mcol(nf, 0.0);
  auto cpos = [&](int j) { return j == nc - 1 ? nf - 1 : 2 * j; };
  for (int k = 0; k < nf; ++k) {
    // M e_k has entries at rows k-1, k, k+1
    std::fill(mcol.begin(), mcol.end(), 0.0);
    if (k > 0) mcol[k - 1] = o.mc[k - 1];
    mcol[k] = o.mb[k];
    if (k + 1 < nf) mcol[k + 1] = o.ma[k + 1];
    // P^T: coarse j gathers fine c_j, and new neighbours with their weights
    for (int j = 0; j < nc; ++j) {
      int c = cpos(j);
      double s = mcol[c];
      if (c >= 2 && (c % 2 == 0)) s += o.rl[j] * mcol[c - 1];
      if (c % 2 == 0 && c < nf - 2) s += o.rr[j] * mcol[c + 1];
      col[j] = s;
    }
    // Thomas solve with the coarse mass matrix
    col[0] = col[0] * o.tr[0];
    for (int i = 1; i < nc; ++i) col[i] = (col[i] - o.ta[i] * col[i - 1]) * o.tr[i];
    for (int i = nc - 2; i >= 0; --i) col[i] = col[i] - o.tcp[i] * col[i + 1];
    for (int j = 0; j < nc; ++j) rows[j] += std::fabs(col[j]);
  }
  double m = 0.0;
  for (double v : rows) m = std::max(m, v);
  return m;
}

DimOps make_ops(const std::vector<double>& x) {
  DimOps o;
  const int nf = (int)x.size();
  const int nc = nf / 2 + 1;
  o.nf = nf;
  o.nc = nc;
  o.wl.assign(nf, 0.0);
  o.wr.assign(nf, 0.0);
  for (int i = 1; i < nf - 1; i += 2) {
    double xl = x[i - 1], xm = x[i], xr = x[i + 1];
    o.wl[i] = (xr - xm) / (xr - xl);
    o.wr[i] = (xm - xl) / (xr - xl);
  }
  mass_bands(x, o.ma, o.mb, o.mc);
  o.rl.assign(nc, 0.0);
  o.rr.assign(nc, 0.0);
  std::vector<double> xc(nc);
  for (int j = 0; j < nc; ++j) {
    int c = j == nc - 1 ? nf - 1 : 2 * j;
    xc[j] = x[c];
    if (c >= 2 && c % 2 == 0) o.rl[j] = o.wr[c - 1];      // new node c-1 weights c by wr
    if (c % 2 == 0 && c < nf - 2) o.rr[j] = o.wl[c + 1];  // new node c+1 weights c by wl
  }
  std::vector<double> b, c;
  mass_bands(xc, o.ta, b, c);
  o.tr.assign(nc, 0.0);
  o.tcp.assign(nc, 0.0);
  o.tr[0] = 1.0 / b[0];
  o.tcp[0] = c[0] * o.tr[0];
  for (int i = 1; i < nc; ++i) {
    o.tr[i] = 1.0 / (b[i] - o.ta[i] * o.tcp[i - 1]);
    o.tcp[i] = c[i] * o.tr[i];
  }
  o.norm_inf = correction_norm(o);
  return o;
}

// W of one level with coordinates x per slot: the product over slots of the
// summed hat integrals (h_left + h_right) / 2 (node counts for slots that are
// not decomposed), minus, for l >= 1 (new_only), the same product over the
// coarse nodes; sums in index order, products in slot order.
void level_weight(const std::array<std::vector<double>, MAXD>& x, const std::array<bool, MAXD>& active,
                  const std::array<int64_t, MAXD>& sizes, bool new_only, double* W) {
  double all_p = 1.0, coarse_p = 1.0;
  for (int s = 0; s < MAXD; ++s) {
    double a = 0.0, c = 0.0;
    if (active[s]) {
      const std::vector<double>& v = x[s];
      const size_t n = v.size();
      for (size_t i = 0; i < n; ++i) {
        const double hl = i > 0 ? v[i] - v[i - 1] : 0.0;
        const double hr = i + 1 < n ? v[i + 1] - v[i] : 0.0;
        a += (hl + hr) / 2.0;
      }
      for (size_t i = 0; i < n; ++i) {
        if (!(i % 2 == 0 || i == n - 1)) continue;
        const double hl = i > 0 ? v[i] - v[i - 1] : 0.0;
        const double hr = i + 1 < n ? v[i + 1] - v[i] : 0.0;
        c += (hl + hr) / 2.0;
      }
    } else {
      a = c = (double)sizes[s];
    }
    all_p *= a;
    coarse_p *= c;
  }
  *W = new_only ? all_p - coarse_p : all_p;
}

std::mutex g_mu;
std::map<std::string, std::shared_ptr<Hierarchy>> g_cache;

}  // namespace

Hierarchy::~Hierarchy() {
  for (int k = 0; k < 2; ++k)
    if (dev_table[k]) (void)hipFree(dev_table[k]);
  if (dev_itab) (void)hipFree(dev_itab);
  if (dev_mass) (void)hipFree(dev_mass);
}

std::shared_ptr<Hierarchy> get_hierarchy(uint32_t ndim, const uint64_t* shape,
                                         const double* const* coords) {
  if (shape == nullptr) fail(MGARD_ERR_ARG, "shape is NULL");
  if (ndim < 1 || ndim > MAXD) fail(MGARD_ERR_SHAPE, "ndim must be 1..4");
  uint64_t total = 1;
  for (uint32_t d = 0; d < ndim; ++d) {
    if (shape[d] == 0) fail(MGARD_ERR_SHAPE, "a side has zero nodes");
    if (shape[d] > (1ull << 31)) fail(MGARD_ERR_SHAPE, "a side exceeds 2^31 nodes");
    total *= shape[d];
    if (total > (1ull << 40)) fail(MGARD_ERR_SHAPE, "more than 2^40 elements");
  }
  std::string key(reinterpret_cast<const char*>(shape), ndim * sizeof(uint64_t));
  for (uint32_t d = 0; d < ndim; ++d) {
    if (coords && coords[d]) {
      for (uint64_t i = 0; i < shape[d]; ++i) {
        if (!std::isfinite(coords[d][i])) fail(MGARD_ERR_ARG, "non-finite coordinate");
        if (i > 0 && !(coords[d][i] > coords[d][i - 1]))
          fail(MGARD_ERR_ARG, "coordinates must be strictly increasing");
      }
      key.push_back('C');
      key.append(reinterpret_cast<const char*>(coords[d]), shape[d] * sizeof(double));
    } else {
      key.push_back('U');
    }
  }
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) return it->second;
  }
  auto h = std::make_shared<Hierarchy>();
  h->D = (int)ndim;
  const int pad = MAXD - (int)ndim;
  std::array<std::vector<double>, MAXD> x;
  int L = -1;
  for (int s = 0; s < MAXD; ++s) {
    int d = s - pad;
    int64_t n = d >= 0 ? (int64_t)shape[d] : 1;
    h->shape[s] = n;
    int k = dim_levels(n);
    h->active[s] = k >= 0;
    if (k >= 0) L = (L < 0) ? k : std::min(L, k);
    x[s].resize(n);
    for (int64_t i = 0; i < n; ++i) x[s][i] = (d >= 0 && coords && coords[d]) ? coords[d][i] : (double)i;
  }
  if (L < 0) L = 0;
  if (L > MAXL - 1) fail(MGARD_ERR_SHAPE, "too many levels");
  h->L = L;
  // the finest grid's mass bands, for the L2 norm of the input
  for (int s = 0; s < MAXD; ++s) {
    if (!h->active[s]) continue;
    std::vector<double> a, b, c;
    mass_bands(x[s], a, b, c);
    h->mass_off[s] = h->mass_table.size();
    h->mass_table.insert(h->mass_table.end(), a.begin(), a.end());
    h->mass_table.insert(h->mass_table.end(), b.begin(), b.end());
    h->mass_table.insert(h->mass_table.end(), c.begin(), c.end());
  }
  if (h->mass_table.empty()) h->mass_table.assign(1, 0.0);
  h->W.assign(L + 1, 0.0);
  h->sizes.assign(L + 1, {});
  h->ops.assign(L + 1, {});
  h->devoff.assign(L + 1, {});
  h->K.assign(L + 1, 0.0);
  for (int s = 0; s < MAXD; ++s) h->sizes[L][s] = h->shape[s];
  for (int l = L; l >= 1; --l) {
    level_weight(x, h->active, h->sizes[l], true, &h->W[l]);
    double k = 1.0;
    for (int s = 0; s < MAXD; ++s) {
      if (!h->active[s]) {
        h->sizes[l - 1][s] = h->sizes[l][s];
        continue;
      }
      DimOps o = make_ops(x[s]);
      k *= o.norm_inf;
      std::vector<double> xc(o.nc);
      for (int j = 0; j < o.nc; ++j) xc[j] = x[s][j == o.nc - 1 ? o.nf - 1 : 2 * j];
      x[s] = std::move(xc);
      h->sizes[l - 1][s] = o.nc;
      h->ops[l][s] = std::move(o);
    }
    h->K[l] = k;
  }
  level_weight(x, h->active, h->sizes[0], false, &h->W[0]);
  double acc = 0.0;
  for (int l = 1; l <= L; ++l) acc += 1.0 + h->K[l];
  h->S = 1.0 + acc;
  // stream layout
  h->level_count.assign(L + 1, 0);
  h->level_off.assign(L + 2, 0);
  h->level_count[0] = h->count(0);
  for (int l = 1; l <= L; ++l) h->level_count[l] = h->count(l) - h->count(l - 1);
  for (int l = 0; l <= L; ++l) h->level_off[l + 1] = h->level_off[l] + h->level_count[l];
  // sub-grid offsets and strides per level (stream positions of new nodes)
  h->itab.assign((uint64_t)(L + 1) * 80, 0);
  for (int l = 1; l <= L; ++l) {
    uint64_t* it = h->itab.data() + 80 * (uint64_t)l;
    uint64_t off = 0;
    for (int m = 1; m < (1 << ndim); ++m) {
      int64_t ext[MAXD];
      for (int s = 0; s < MAXD; ++s) {
        const int d = s - pad;
        const bool bit = d >= 0 && ((m >> d) & 1);
        ext[s] = bit ? (h->sizes[l][s] - h->sizes[l - 1][s]) : h->sizes[l - 1][s];
      }
      uint64_t acc = 1;
      for (int s = MAXD - 1; s >= 0; --s) {
        it[16 + 4 * m + s] = acc;
        acc *= (uint64_t)ext[s];
      }
      it[m] = off;
      off += acc;
    }
  }
  // constant table
  auto& t = h->table;
  auto put = [&](const std::vector<double>& v) {
    uint64_t off = t.size();
    t.insert(t.end(), v.begin(), v.end());
    while (t.size() % 64) t.push_back(0.0);  // keep arrays 256-byte aligned in float64
    return off;
  };
  for (int l = 1; l <= L; ++l)
    for (int s = 0; s < MAXD; ++s) {
      if (!h->active[s]) continue;
      const DimOps& o = h->ops[l][s];
      DevDim& dd = h->devoff[l][s];
      dd.wl = put(o.wl);
      dd.wr = put(o.wr);
      dd.ma = put(o.ma);
      dd.mb = put(o.mb);
      dd.mc = put(o.mc);
      dd.rl = put(o.rl);
      dd.rr = put(o.rr);
      dd.ta = put(o.ta);
      dd.tr = put(o.tr);
      dd.tcp = put(o.tcp);
    }
  if (t.empty()) t.assign(64, 0.0);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    if (g_cache.size() > 1024) g_cache.clear();
    g_cache[key] = h;
  }
  return h;
}

const void* device_table(Hierarchy& h, bool f64, hipStream_t stream) {
  int dev = 0;
  MG_HIP(hipGetDevice(&dev));
  const int k = f64 ? 1 : 0;
  std::lock_guard<std::mutex> lk(g_mu);
  if (!h.dev_itab || h.dev_itab_id != dev) {
    if (h.dev_itab) (void)hipFree(h.dev_itab);
    h.dev_itab = nullptr;
    if (hipMalloc(&h.dev_itab, h.itab.size() * 8) != hipSuccess) fail(MGARD_ERR_OOM, "sub-grid table");
    MG_HIP(hipMemcpyAsync(h.dev_itab, h.itab.data(), h.itab.size() * 8, hipMemcpyHostToDevice, stream));
    MG_HIP(hipStreamSynchronize(stream));
    h.dev_itab_id = dev;
  }
  if (h.dev_table[k] && h.dev_id[k] == dev) return h.dev_table[k];
  if (h.dev_table[k]) {
    (void)hipFree(h.dev_table[k]);
    h.dev_table[k] = nullptr;
  }
  const size_t n = h.table.size();
  void* p = nullptr;
  if (hipMalloc(&p, n * (f64 ? 8 : 4)) != hipSuccess) fail(MGARD_ERR_OOM, "constant table");
  if (f64) {
    MG_HIP(hipMemcpyAsync(p, h.table.data(), n * 8, hipMemcpyHostToDevice, stream));
  } else {
    std::vector<float> f(n);
    for (size_t i = 0; i < n; ++i) f[i] = static_cast<float>(h.table[i]);
    MG_HIP(hipMemcpyAsync(p, f.data(), n * 4, hipMemcpyHostToDevice, stream));
  }
  MG_HIP(hipStreamSynchronize(stream));
  h.dev_table[k] = p;
  h.dev_id[k] = dev;
  return p;
}

const double* device_mass_table(Hierarchy& h, hipStream_t stream) {
  int dev = 0;
  MG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_mu);
  if (h.dev_mass && h.dev_mass_id == dev) return static_cast<const double*>(h.dev_mass);
  if (h.dev_mass) (void)hipFree(h.dev_mass);
  h.dev_mass = nullptr;
  void* p = nullptr;
  if (hipMalloc(&p, h.mass_table.size() * 8) != hipSuccess) fail(MGARD_ERR_OOM, "mass table");
  MG_HIP(hipMemcpyAsync(p, h.mass_table.data(), h.mass_table.size() * 8, hipMemcpyHostToDevice, stream));
  MG_HIP(hipStreamSynchronize(stream));
  h.dev_mass = p;
  h.dev_mass_id = dev;
  return static_cast<const double*>(p);
}

// ----------------------------------------------------------------- workspace
void Workspace::reserve(uint64_t bytes) {
  if (bytes <= size_) return;
  if (base_) {
    MG_HIP(hipDeviceSynchronize());
    (void)hipFree(base_);
    base_ = nullptr;
    size_ = 0;
  }
  uint64_t want = bytes + bytes / 8 + (1 << 20);
  if (hipMalloc(&base_, want) != hipSuccess) {
    (void)hipGetLastError();
    base_ = nullptr;
    fail(MGARD_ERR_OOM, "workspace of " + std::to_string(want) + " bytes");
  }
  size_ = want;
}

void Workspace::release() {
  if (base_) {
    (void)hipDeviceSynchronize();
    (void)hipFree(base_);
  }
  base_ = nullptr;
  size_ = 0;
}

Workspace& workspace() {
  static Workspace ws[64];
  int dev = 0;
  MG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) fail(MGARD_ERR_DEVICE, "device index");
  return ws[dev];
}

uint8_t* pinned_staging(size_t bytes) {
  thread_local uint8_t* p = nullptr;
  thread_local size_t cap = 0;
  if (bytes > cap) {
    // only between calls (every call that stages waits for its copies)
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    void* q = nullptr;
    const size_t n = std::max<size_t>(bytes, 65536);
    if (hipHostMalloc(&q, n, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      fail(MGARD_ERR_OOM, "pinned staging");
    }
    p = static_cast<uint8_t*>(q);
    cap = n;
  }
  return p;
}

Workspace& aux_workspace() {
  static Workspace ws[64];
  int dev = 0;
  MG_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) fail(MGARD_ERR_DEVICE, "device index");
  return ws[dev];
}

}  // namespace mg
