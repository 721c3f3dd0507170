// FP64 oracle, raster half: tile binning and depth sort, front-to-back compositing
// (Eq. 1), its adjoint, a brute-force compositor and the photometric loss (Eq. 3).
// Test infrastructure only (see oracle.h).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <numeric>
#include <thread>
#include <vector>

#include "oracle.h"

namespace {

int g_threads = 0;

int threads() {
  if (g_threads > 0) return g_threads;
  const char* e = std::getenv("ORC_THREADS");
  if (e && std::atoi(e) > 0) return std::atoi(e);
  unsigned h = std::thread::hardware_concurrency();
  return h ? (int)h : 1;
}

// Runs body(lo, hi, worker) over [0, n) split into contiguous chunks.
void parallel_for(int n, const std::function<void(int, int, int)>& body) {
  const int T = std::max(1, std::min(threads(), n));
  if (T == 1) { body(0, n, 0); return; }
  std::vector<std::thread> th;
  for (int w = 0; w < T; ++w) {
    const int lo = (int)((long)n * w / T), hi = (int)((long)n * (w + 1) / T);
    th.emplace_back(body, lo, hi, w);
  }
  for (auto& t : th) t.join();
}

const double kAlphaMin = 1.0 / 255.0;  // skip threshold
const double kAlphaMax = 0.99;         // alpha clamp
const double kTMin = 1e-4;             // transmittance stop threshold

// Widths of the ambiguity windows (parity bookkeeping only; no effect on any value).
struct Margins {
  double alpha = 1e-6;   // |alpha - 1/255|
  double T = 1e-8;       // |T' - 1e-4|
  double depth = 1e-6;   // relative depth gap of two entries that take part
  double clamp = 1e-6;   // |raw alpha - 0.99|
};
Margins g_margin;

// When set, the compositing adjoint accumulates the magnitude of every term instead of
// the term (each factor replaced by its absolute value): the sum of |terms| an element
// is formed from, the scale of its floating-point rounding error.
bool g_magnitude = false;

// One Gaussian evaluated at a pixel centre.
struct Eval {
  double dx, dy;   // u - (x + 0.5), v - (y + 0.5)
  double power;    // -(A dx^2 + C dy^2)/2 - B dx dy
  double ep;       // exp(power)
  double raw;      // opacity * exp(power)
  double alpha;    // min(0.99, raw)
};

Eval evaluate(double u, double v, const double con[3], double op, int x, int y) {
  Eval e;
  e.dx = u - (x + 0.5);
  e.dy = v - (y + 0.5);
  e.power = -0.5 * (con[0] * e.dx * e.dx + con[2] * e.dy * e.dy) - con[1] * e.dx * e.dy;
  e.ep = std::exp(e.power);
  e.raw = op * e.ep;
  e.alpha = std::min(kAlphaMax, e.raw);
  return e;
}

struct Contribution {
  int g;          // Gaussian
  double T;       // transmittance in front of it
  Eval e;
};

struct PixelResult {
  double C[3];
  double T;
  int n_contrib;  // 1 + list position of the last composited entry
  int n_eval;     // entries visited up to and including the stopping one
  uint8_t amb;
  std::vector<Contribution> list;
};

// Front-to-back compositing of an ordered entry list at pixel (x, y), Eq. 1:
// C = sum_i c_i a_i prod_{j<i}(1 - a_j), with the readings: alpha clamped to 0.99,
// entries with alpha < 1/255 skipped, and the walk stopped before an entry that would
// take the transmittance below 1e-4.  `cand(i)` says whether entry i is a candidate
// (its footprint box holds the pixel); non-candidates are only checked for ambiguity.
template <class GetG, class IsCand>
void composite(int n, GetG getg, IsCand cand, const double* uv, const double* conic,
               const double* opacity, const double* rgb, const double* depth, int G, int x,
               int y, const double* bg, PixelResult& r) {
  r.C[0] = r.C[1] = r.C[2] = 0.0;
  r.T = 1.0;
  r.n_contrib = 0;
  r.n_eval = n;
  r.amb = 0;
  r.list.clear();
  double prev_depth = -1.0;
  for (int i = 0; i < n; ++i) {
    const int g = getg(i);
    const double con[3] = {conic[g], conic[(size_t)G + g], conic[2 * (size_t)G + g]};
    const Eval e = evaluate(uv[g], uv[(size_t)G + g], con, opacity[g], x, y);
    if (!cand(i)) {
      if (e.alpha > kAlphaMin - g_margin.alpha) r.amb |= ORC_AMB_ALPHA;
      continue;
    }
    if (std::fabs(e.alpha - kAlphaMin) < g_margin.alpha) r.amb |= ORC_AMB_ALPHA;
    if (std::fabs(e.raw - kAlphaMax) < g_margin.clamp) r.amb |= ORC_AMB_CLAMP;
    if (e.alpha < kAlphaMin) continue;
    // an order flip between two entries that both take part changes the pixel
    if (prev_depth >= 0.0 && std::fabs(depth[g] - prev_depth) < g_margin.depth * depth[g])
      r.amb |= ORC_AMB_DEPTH;
    prev_depth = depth[g];
    const double Tn = r.T * (1.0 - e.alpha);
    if (std::fabs(Tn - kTMin) < g_margin.T) r.amb |= ORC_AMB_T;
    if (Tn < kTMin) {
      r.n_eval = i + 1;
      // the stopping entry swapped with a near-tie that follows it changes which of
      // the two is composited: look ahead over the entries of equal depth
      for (int j = i + 1; j < n; ++j) {
        const int h = getg(j);
        if (std::fabs(depth[h] - depth[g]) >= g_margin.depth * depth[g]) break;
        if (!cand(j)) continue;
        const double ch[3] = {conic[h], conic[(size_t)G + h], conic[2 * (size_t)G + h]};
        if (evaluate(uv[h], uv[(size_t)G + h], ch, opacity[h], x, y).alpha > kAlphaMin - g_margin.alpha)
          r.amb |= ORC_AMB_DEPTH;
      }
      break;
    }
    for (int c = 0; c < 3; ++c) r.C[c] += rgb[c * (size_t)G + g] * e.alpha * r.T;
    r.list.push_back({g, r.T, e});
    r.T = Tn;
    r.n_contrib = i + 1;
  }
  for (int c = 0; c < 3; ++c) r.C[c] += r.T * bg[c];
}

// The composited lists of one image row (orc_render_lists).
struct PixelLists {
  std::vector<int64_t> count;
  std::vector<int32_t> ids;
  std::vector<uint8_t> clamped;
};

bool in_rect(const int32_t* prect, int G, int g, int x, int y) {
  return x >= prect[g] && x <= prect[(size_t)G + g] && y >= prect[2 * (size_t)G + g] &&
         y <= prect[3 * (size_t)G + g];
}

// Gradient of one pixel's colour with respect to the 2-D parameters of its composited
// Gaussians, using the stored forward transmittances:
//   dC/dc_i = a_i T_i
//   dC/da_i = c_i T_i - (sum_{j>i} c_j a_j T_j + T_final bg) / (1 - a_i)
//   da_i/dopacity = exp(power), da_i/dpower = a_i   (zero when the 0.99 clamp is active)
//   power = -(A dx^2 + C dy^2)/2 - B dx dy with dx = u - x - 1/2, dy = v - y - 1/2.
void pixel_backward_magnitude(const PixelResult& r, const double* rgb, const double* conic,
                              int G, const double* bg, const double g[3], double* acc);

void pixel_backward(const PixelResult& r, const double* rgb, const double* conic, int G,
                    const double* bg, const double g[3], double* acc /*[9][G]*/) {
  if (g_magnitude) {
    pixel_backward_magnitude(r, rgb, conic, G, bg, g, acc);
    return;
  }
  const int n = (int)r.list.size();
  double behind[3] = {r.T * bg[0], r.T * bg[1], r.T * bg[2]};
  for (int i = n - 1; i >= 0; --i) {
    const Contribution& k = r.list[i];
    const int id = k.g;
    const double a = k.e.alpha, T = k.T;
    double dL_da = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double col = rgb[c * (size_t)G + id];
      acc[(6 + c) * (size_t)G + id] += g[c] * a * T;
      dL_da += g[c] * (col * T - behind[c] / (1.0 - a));
    }
    for (int c = 0; c < 3; ++c) behind[c] += rgb[c * (size_t)G + id] * a * T;
    if (k.e.raw > kAlphaMax) continue;  // clamped: alpha does not depend on its inputs
    acc[5 * (size_t)G + id] += dL_da * k.e.ep;
    const double dp = dL_da * a;
    const double A = conic[id], B = conic[(size_t)G + id], C = conic[2 * (size_t)G + id];
    const double dx = k.e.dx, dy = k.e.dy;
    acc[0 * (size_t)G + id] += dp * (-(A * dx + B * dy));
    acc[1 * (size_t)G + id] += dp * (-(B * dx + C * dy));
    acc[2 * (size_t)G + id] += dp * (-0.5 * dx * dx);
    acc[3 * (size_t)G + id] += dp * (-dx * dy);
    acc[4 * (size_t)G + id] += dp * (-0.5 * dy * dy);
  }
}

// The same terms as pixel_backward with every factor taken by magnitude: for each of
// the nine elements, the sum of |term| over this pixel's contributions.
void pixel_backward_magnitude(const PixelResult& r, const double* rgb, const double* conic,
                              int G, const double* bg, const double g[3], double* acc) {
  const int n = (int)r.list.size();
  double behind[3] = {r.T * std::fabs(bg[0]), r.T * std::fabs(bg[1]), r.T * std::fabs(bg[2])};
  for (int i = n - 1; i >= 0; --i) {
    const Contribution& k = r.list[i];
    const int id = k.g;
    const double a = k.e.alpha, T = k.T;
    double dL_da = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double col = std::fabs(rgb[c * (size_t)G + id]);
      acc[(6 + c) * (size_t)G + id] += std::fabs(g[c]) * a * T;
      dL_da += std::fabs(g[c]) * (col * T + behind[c] / (1.0 - a));
    }
    for (int c = 0; c < 3; ++c) behind[c] += std::fabs(rgb[c * (size_t)G + id]) * a * T;
    if (k.e.raw > kAlphaMax) continue;
    acc[5 * (size_t)G + id] += dL_da * k.e.ep;
    const double dp = dL_da * a;
    const double A = std::fabs(conic[id]), B = std::fabs(conic[(size_t)G + id]),
                 C = std::fabs(conic[2 * (size_t)G + id]);
    const double dx = std::fabs(k.e.dx), dy = std::fabs(k.e.dy);
    acc[0 * (size_t)G + id] += dp * (A * dx + B * dy);
    acc[1 * (size_t)G + id] += dp * (B * dx + C * dy);
    acc[2 * (size_t)G + id] += dp * (0.5 * dx * dx);
    acc[3 * (size_t)G + id] += dp * (dx * dy);
    acc[4 * (size_t)G + id] += dp * (0.5 * dy * dy);
  }
}

// Brute-force candidate list of a pixel: every visible Gaussian whose footprint box
// holds it, ordered by (depth, index).
void brute_list(int G, const int32_t* prect, const double* depth, int x, int y,
                std::vector<int>& ids) {
  ids.clear();
  for (int g = 0; g < G; ++g)
    if (in_rect(prect, G, g, x, y)) ids.push_back(g);
  std::stable_sort(ids.begin(), ids.end(), [&](int a, int b) { return depth[a] < depth[b]; });
}

}  // namespace

extern "C" {

int orc_num_threads(void) { return threads(); }
void orc_set_num_threads(int n) { g_threads = n; }

void orc_set_margins(double alpha, double T, double depth, double clamp) {
  g_margin.alpha = alpha;
  g_margin.T = T;
  g_margin.depth = depth;
  g_margin.clamp = clamp;
}

void orc_set_magnitude_mode(int on) { g_magnitude = on != 0; }

void orc_bin_sort(int n_views, const int64_t* gbegin, const int32_t* tiles_x,
                  const int32_t* tiles_y, const int64_t* tile_base, int tile_w, int tile_h,
                  const int32_t* prect, const double* depth, int64_t G, int64_t T_total,
                  int32_t* tile, int32_t* vals, int64_t* ranges) {
  (void)tiles_y;
  struct Pair {
    int64_t tile;
    double depth;
    int32_t val;
  };
  std::vector<Pair> pairs;
  for (int k = 0; k < n_views; ++k) {
    for (int64_t g = gbegin[k]; g < gbegin[k + 1]; ++g) {
      const int x0 = prect[g], x1 = prect[G + g], y0 = prect[2 * G + g], y1 = prect[3 * G + g];
      if (x0 > x1 || y0 > y1) continue;
      for (int ty = y0 / tile_h; ty <= y1 / tile_h; ++ty)
        for (int tx = x0 / tile_w; tx <= x1 / tile_w; ++tx)
          pairs.push_back({tile_base[k] + (int64_t)ty * tiles_x[k] + tx, depth[g], (int32_t)g});
    }
  }
  std::stable_sort(pairs.begin(), pairs.end(), [](const Pair& a, const Pair& b) {
    return a.tile != b.tile ? a.tile < b.tile : a.depth < b.depth;
  });
  for (int64_t t = 0; t < T_total; ++t) ranges[2 * t] = ranges[2 * t + 1] = 0;
  for (size_t i = 0; i < pairs.size(); ++i) {
    tile[i] = (int32_t)pairs[i].tile;
    vals[i] = pairs[i].val;
    const int64_t t = pairs[i].tile;
    if (i == 0 || pairs[i - 1].tile != t) ranges[2 * t] = (int64_t)i;
    if (i + 1 == pairs.size() || pairs[i + 1].tile != t) ranges[2 * t + 1] = (int64_t)i + 1;
  }
}

void orc_render_fwd(int G, const double* uv, const double* conic, const double* opacity,
                    const double* rgb, const int32_t* prect, const double* depth,
                    const int32_t* vals, const int64_t* ranges, int W, int H, int tile_w,
                    int tile_h, const double* bg, double* image, double* T_final,
                    int32_t* n_contrib, int32_t* n_eval, uint8_t* amb) {
  const int tiles_x = (W + tile_w - 1) / tile_w;
  const size_t HW = (size_t)H * W;
  parallel_for(H, [&](int lo, int hi, int) {
    PixelResult r;
    for (int y = lo; y < hi; ++y)
      for (int x = 0; x < W; ++x) {
        const int t = (y / tile_h) * tiles_x + x / tile_w;
        const int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
        composite((int)(e - s), [&](int i) { return vals[s + i]; },
                  [&](int i) { return in_rect(prect, G, vals[s + i], x, y); }, uv, conic, opacity,
                  rgb, depth, G, x, y, bg, r);
        const size_t p = (size_t)y * W + x;
        for (int c = 0; c < 3; ++c) image[c * HW + p] = r.C[c];
        T_final[p] = r.T;
        n_contrib[p] = r.n_contrib;
        n_eval[p] = r.n_eval;
        amb[p] = r.amb;
      }
  });
}

void orc_render_bwd(int G, const double* uv, const double* conic, const double* opacity,
                    const double* rgb, const int32_t* prect, const double* depth,
                    const int32_t* vals, const int64_t* ranges, int W, int H, int tile_w,
                    int tile_h, const double* bg, const double* dimage, double* g2d) {
  const int tiles_x = (W + tile_w - 1) / tile_w;
  const size_t HW = (size_t)H * W;
  const int T = std::max(1, std::min(threads(), H));
  std::vector<std::vector<double>> part(T);
  parallel_for(H, [&](int lo, int hi, int w) {
    std::vector<double>& acc = part[w];
    acc.assign((size_t)9 * G, 0.0);
    PixelResult r;
    for (int y = lo; y < hi; ++y)
      for (int x = 0; x < W; ++x) {
        const int t = (y / tile_h) * tiles_x + x / tile_w;
        const int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
        composite((int)(e - s), [&](int i) { return vals[s + i]; },
                  [&](int i) { return in_rect(prect, G, vals[s + i], x, y); }, uv, conic, opacity,
                  rgb, depth, G, x, y, bg, r);
        const size_t p = (size_t)y * W + x;
        const double gp[3] = {dimage[p], dimage[HW + p], dimage[2 * HW + p]};
        pixel_backward(r, rgb, conic, G, bg, gp, acc.data());
      }
  });
  for (size_t i = 0; i < (size_t)9 * G; ++i) {
    double s = 0.0;
    for (int w = 0; w < T; ++w)
      if (!part[w].empty()) s += part[w][i];
    g2d[i] = s;
  }
}

void* orc_render_lists(int G, const double* uv, const double* conic, const double* opacity,
                       const double* rgb, const int32_t* prect, const double* depth,
                       const int32_t* vals, const int64_t* ranges, int W, int H, int tile_w,
                       int tile_h, int64_t* total) {
  const int tiles_x = (W + tile_w - 1) / tile_w;
  const double bg[3] = {0.0, 0.0, 0.0};
  auto* rows = new std::vector<PixelLists>(H);
  parallel_for(H, [&](int lo, int hi, int) {
    PixelResult r;
    for (int y = lo; y < hi; ++y) {
      PixelLists& row = (*rows)[y];
      row.count.assign(W, 0);
      for (int x = 0; x < W; ++x) {
        const int t = (y / tile_h) * tiles_x + x / tile_w;
        const int64_t s = ranges[2 * t], e = ranges[2 * t + 1];
        composite((int)(e - s), [&](int i) { return vals[s + i]; },
                  [&](int i) { return in_rect(prect, G, vals[s + i], x, y); }, uv, conic, opacity,
                  rgb, depth, G, x, y, bg, r);
        row.count[x] = (int64_t)r.list.size();
        for (const Contribution& k : r.list) {
          row.ids.push_back(k.g);
          row.clamped.push_back(k.e.raw > kAlphaMax ? 1 : 0);
        }
      }
    }
  });
  int64_t n = 0;
  for (const PixelLists& row : *rows) n += (int64_t)row.ids.size();
  *total = n;
  return rows;
}

void orc_render_lists_take(void* handle, int64_t* offsets, int32_t* ids, uint8_t* clamped) {
  auto* rows = static_cast<std::vector<PixelLists>*>(handle);
  int64_t o = 0;
  size_t p = 0;
  offsets[0] = 0;
  for (const PixelLists& row : *rows) {
    for (int64_t c : row.count) offsets[++p] = (o += c);
    std::copy(row.ids.begin(), row.ids.end(), ids + (o - (int64_t)row.ids.size()));
    std::copy(row.clamped.begin(), row.clamped.end(), clamped + (o - (int64_t)row.ids.size()));
  }
  delete rows;
}

void orc_render_frozen(int G, const double* uv, const double* conic, const double* opacity,
                       const double* rgb, int W, int H, const double* bg,
                       const int64_t* offsets, const int32_t* ids, const uint8_t* clamped,
                       double* image, double* T_final) {
  const size_t HW = (size_t)H * W;
  parallel_for(H, [&](int lo, int hi, int) {
    for (int y = lo; y < hi; ++y)
      for (int x = 0; x < W; ++x) {
        const size_t p = (size_t)y * W + x;
        double C[3] = {0.0, 0.0, 0.0}, T = 1.0;
        for (int64_t o = offsets[p]; o < offsets[p + 1]; ++o) {
          const int g = ids[o];
          const double con[3] = {conic[g], conic[(size_t)G + g], conic[2 * (size_t)G + g]};
          const Eval e = evaluate(uv[g], uv[(size_t)G + g], con, opacity[g], x, y);
          const double a = clamped[o] ? kAlphaMax : e.raw;
          for (int c = 0; c < 3; ++c) C[c] += rgb[c * (size_t)G + g] * a * T;
          T *= 1.0 - a;
        }
        for (int c = 0; c < 3; ++c) image[c * HW + p] = C[c] + T * bg[c];
        T_final[p] = T;
      }
  });
}

void orc_render_brute(int G, const double* uv, const double* conic, const double* opacity,
                      const double* rgb, const int32_t* prect, const double* depth, int W,
                      int H, const double* bg, double* image, double* T_final,
                      int32_t* n_contrib, uint8_t* amb) {
  const size_t HW = (size_t)H * W;
  parallel_for(H, [&](int lo, int hi, int) {
    PixelResult r;
    std::vector<int> ids;
    for (int y = lo; y < hi; ++y)
      for (int x = 0; x < W; ++x) {
        brute_list(G, prect, depth, x, y, ids);
        composite((int)ids.size(), [&](int i) { return ids[i]; }, [](int) { return true; }, uv,
                  conic, opacity, rgb, depth, G, x, y, bg, r);
        const size_t p = (size_t)y * W + x;
        for (int c = 0; c < 3; ++c) image[c * HW + p] = r.C[c];
        T_final[p] = r.T;
        n_contrib[p] = r.n_contrib;
        amb[p] = r.amb;
      }
  });
}

void orc_render_brute_bwd(int G, const double* uv, const double* conic,
                          const double* opacity, const double* rgb, const int32_t* prect,
                          const double* depth, int W, int H, const double* bg,
                          const double* dimage, double* g2d) {
  const size_t HW = (size_t)H * W;
  std::fill(g2d, g2d + (size_t)9 * G, 0.0);
  PixelResult r;
  std::vector<int> ids;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      brute_list(G, prect, depth, x, y, ids);
      composite((int)ids.size(), [&](int i) { return ids[i]; }, [](int) { return true; }, uv,
                conic, opacity, rgb, depth, G, x, y, bg, r);
      const size_t p = (size_t)y * W + x;
      const double gp[3] = {dimage[p], dimage[HW + p], dimage[2 * HW + p]};
      const int n = (int)r.list.size();
      // alphas of the composited list; the stop decision is a discrete choice that
      // does not move under a small change, so the list is held fixed
      std::vector<double> a(n);
      for (int i = 0; i < n; ++i) a[i] = r.list[i].e.alpha;
      for (int i = 0; i < n; ++i) {
        const int id = r.list[i].g;
        // prod_{j<i} (1 - a_j)
        double Ti = 1.0;
        for (int j = 0; j < i; ++j) Ti *= 1.0 - a[j];
        double dL_da = 0.0;
        for (int c = 0; c < 3; ++c) {
          const double col = rgb[c * (size_t)G + id];
          g2d[(6 + c) * (size_t)G + id] += gp[c] * a[i] * Ti;
          // derivative of sum_k c_k a_k prod_{j<k}(1 - a_j) + bg prod_j (1 - a_j)
          double d = col * Ti;
          for (int k = i + 1; k < n; ++k) {
            double prod = 1.0;
            for (int j = 0; j < k; ++j)
              if (j != i) prod *= 1.0 - a[j];
            d -= rgb[c * (size_t)G + r.list[k].g] * a[k] * prod;
          }
          double prod_all = 1.0;
          for (int j = 0; j < n; ++j)
            if (j != i) prod_all *= 1.0 - a[j];
          d -= bg[c] * prod_all;
          dL_da += gp[c] * d;
        }
        const Eval& e = r.list[i].e;
        if (e.raw > kAlphaMax) continue;
        g2d[5 * (size_t)G + id] += dL_da * e.ep;
        const double dp = dL_da * e.alpha;
        const double A = conic[id], B = conic[(size_t)G + id], C = conic[2 * (size_t)G + id];
        g2d[0 * (size_t)G + id] += dp * (-(A * e.dx + B * e.dy));
        g2d[1 * (size_t)G + id] += dp * (-(B * e.dx + C * e.dy));
        g2d[2 * (size_t)G + id] += dp * (-0.5 * e.dx * e.dx);
        g2d[3 * (size_t)G + id] += dp * (-e.dx * e.dy);
        g2d[4 * (size_t)G + id] += dp * (-0.5 * e.dy * e.dy);
      }
    }
}

double orc_loss_signed(int W, int H, const double* image, const double* target, double w_ssim,
                       const double* l1_sign, double* loss_px, double* ssim, double* dimage);

double orc_loss(int W, int H, const double* image, const double* target, double w_ssim,
                double* loss_px, double* ssim, double* dimage) {
  return orc_loss_signed(W, H, image, target, w_ssim, nullptr, loss_px, ssim, dimage);
}

double orc_loss_signed(int W, int H, const double* image, const double* target, double w_ssim,
                       const double* l1_sign, double* loss_px, double* ssim, double* dimage) {
  const size_t HW = (size_t)H * W;
  const double n = 3.0 * (double)HW;
  const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
  const int R = 5;  // 11x11 window
  const double inv_win = 1.0 / 121.0;
  for (size_t p = 0; p < HW; ++p) loss_px[p] = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double* x = image + c * HW;
    const double* y = target + c * HW;
    double* dx = dimage + c * HW;
    // L1 term: sign(0) = 0
    for (size_t p = 0; p < HW; ++p) {
      const double d = x[p] - y[p];
      const double sg = l1_sign ? l1_sign[c * HW + p] : (d > 0.0 ? 1.0 : (d < 0.0 ? -1.0 : 0.0));
      loss_px[p] += sg * d / n;
      dx[p] = sg / n;
    }
    if (w_ssim == 0.0) {
      for (size_t p = 0; p < HW; ++p) ssim[c * HW + p] = 1.0;
      continue;
    }
    // window statistics with zero padding: means over the 11x11 box, divisor 121
    std::vector<double> ds_dmx(HW), ds_dexx(HW), ds_dexy(HW);
    parallel_for(H, [&](int lo, int hi, int) {
      for (int qy = lo; qy < hi; ++qy)
        for (int qx = 0; qx < W; ++qx) {
          double sx = 0, sy = 0, sxx = 0, syy = 0, sxy = 0;
          for (int oy = -R; oy <= R; ++oy)
            for (int ox = -R; ox <= R; ++ox) {
              const int px = qx + ox, py = qy + oy;
              if (px < 0 || px >= W || py < 0 || py >= H) continue;
              const double a = x[(size_t)py * W + px], b = y[(size_t)py * W + px];
              sx += a; sy += b; sxx += a * a; syy += b * b; sxy += a * b;
            }
          const double mx = sx * inv_win, my = sy * inv_win;
          const double exx = sxx * inv_win, eyy = syy * inv_win, exy = sxy * inv_win;
          const double vx = exx - mx * mx, vy = eyy - my * my, cxy = exy - mx * my;
          const double n1 = 2 * mx * my + C1, n2 = 2 * cxy + C2;
          const double d1 = mx * mx + my * my + C1, d2 = vx + vy + C2;
          const double s = (n1 * n2) / (d1 * d2);
          const size_t q = (size_t)qy * W + qx;
          ssim[c * HW + q] = s;
          // partial derivatives of s with respect to mean(x), E[x^2], E[xy]
          // (var(x) = E[x^2] - mean(x)^2, cov = E[xy] - mean(x) mean(y))
          const double dn1 = 2 * my, dn2 = -2 * my, dd1 = 2 * mx, dd2 = -2 * mx;
          ds_dmx[q] = (dn1 * n2 + n1 * dn2) / (d1 * d2) - s * (dd1 * d2 + d1 * dd2) / (d1 * d2);
          ds_dexx[q] = -s / d2;
          ds_dexy[q] = 2 * n1 / (d1 * d2);
        }
    });
    for (size_t q = 0; q < HW; ++q) loss_px[q] += w_ssim * (1.0 - ssim[c * HW + q]) / n;
    // adjoint of the window means: pixel p feeds every window q within 5 of it
    parallel_for(H, [&](int lo, int hi, int) {
      for (int py = lo; py < hi; ++py)
        for (int px = 0; px < W; ++px) {
          const size_t p = (size_t)py * W + px;
          double acc = 0.0;
          for (int oy = -R; oy <= R; ++oy)
            for (int ox = -R; ox <= R; ++ox) {
              const int qx = px + ox, qy = py + oy;
              if (qx < 0 || qx >= W || qy < 0 || qy >= H) continue;
              const size_t q = (size_t)qy * W + qx;
              acc += ds_dmx[q] + 2.0 * x[p] * ds_dexx[q] + y[p] * ds_dexy[q];
            }
          dx[p] += -w_ssim * acc * inv_win / n;
        }
    });
  }
  double L = 0.0;
  for (size_t p = 0; p < HW; ++p) L += loss_px[p];
  return L;
}

}  // extern "C"
