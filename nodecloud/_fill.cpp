// Seeded node placement for one periodic simple-cubic cell of side 1 holding a
// sphere of radius r centred at (1/2, 1/2, 1/2); for r > 1/2 the sphere and its
// periodic images overlap.  This is input preparation only: it places nodes and
// holds none of the solver arithmetic.
//
// Boundary nodes: a Fibonacci lattice on the sphere under a seeded random
// rotation, one point per 1.15*hb^2 of surface (the density that reproduces
// the paper's count of about 175 surface nodes for r = 0.04 at h_min = 0.01,
// Sec. 3.4); a point is kept only if it lies inside the
// cell, which drops the parts of the sphere that are covered by its images,
// and only if no surface point placed before it lies within half the surface
// spacing (near the circles where the grain meets its images).
// Each boundary node carries the unit normal pointing from the solid into the
// fluid.
//
// Interior nodes: an advancing front seeded with the boundary nodes (in the
// spirit of the dimension-independent variable-density generator the paper
// uses, Sec. 2.1).  A dequeued node x_d spawns n_cand candidates on a sphere of
// radius h(x_d); a candidate is kept if it is in the fluid, at least half its
// spacing away from the wall, and no existing node
// lies closer than min(h(candidate), h(x_d)) under the minimum-image
// convention.  The target spacing h(d), d the distance to the grain, is either
// linear, h(d) = min(h0 + slope*d, hmax), or the paper's Gaussian refinement
// (Sec. 2.4, Eq. refinement_function), h = hmax - exp(-t^2 / (2 eps^2))
// (hmax - hmin) with t = d / (sqrt(3)/2 - r): the distance normalised by the
// largest distance from a grain that the cell holds (the printed product form
// is read as this quotient, which the paper's node counts fit).
//
// Build: g++ -O2 -shared -fPIC _fill.cpp -o _libfill.so
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

struct Rng {  // xoshiro256** seeded through splitmix64
  uint64_t s[4];
  explicit Rng(uint64_t seed) {
    uint64_t z = seed + 0x9E3779B97F4A7C15ull;
    for (int i = 0; i < 4; ++i) {
      z += 0x9E3779B97F4A7C15ull;
      uint64_t x = z;
      x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
      x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
      s[i] = x ^ (x >> 31);
    }
  }
  static uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
  uint64_t next() {
    uint64_t r = rotl(s[1] * 5, 7) * 9, t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3]; s[2] ^= t; s[3] = rotl(s[3], 45);
    return r;
  }
  double uniform() { return (next() >> 11) * (1.0 / 9007199254740992.0); }
  void unit(double* u) {  // uniform direction on the unit sphere
    double z = 2.0 * uniform() - 1.0, ph = 2.0 * M_PI * uniform();
    double rho = std::sqrt(std::fmax(0.0, 1.0 - z * z));
    u[0] = rho * std::cos(ph); u[1] = rho * std::sin(ph); u[2] = z;
  }
};

inline double wrap(double x) {
  x -= std::floor(x);
  return x >= 1.0 ? 0.0 : x;
}
inline double mi(double d) { return d - std::nearbyint(d); }

struct Spacing {  // target internodal distance as a function of the distance d to the grain
  int gaussian;
  double a, b, c;  // linear: h0, slope, hmax; Gaussian: hmin, hmax, eps
  double norm;     // Gaussian: sqrt(3)/2 - r
  double operator()(double d) const {
    d = std::fmax(d, 0.0);
    if (!gaussian) return std::fmin(a + b * d, c);
    const double t = d / norm;
    return b - std::exp(-t * t / (2.0 * c * c)) * (b - a);
  }
  double lo() const { return a; }
  double hi() const { return gaussian ? b : c; }
};

struct Cell {
  double r;
  double sdf(const double* x) const {
    double dx = mi(x[0] - 0.5), dy = mi(x[1] - 0.5), dz = mi(x[2] - 0.5);
    return std::sqrt(dx * dx + dy * dy + dz * dz) - r;
  }
};

// Multi-level hashed cell lists.  Level l has cells of side >= hmin * 2^l; a
// radius query uses the finest level whose cell side is not below the radius,
// so it scans 27 cells.  Hash collisions merge lists, which only costs extra
// distance tests.
struct Grid {
  struct Level { int g; double inv; std::vector<int32_t> head; };
  std::vector<Level> lv;
  std::vector<std::vector<int32_t>> next;
  uint64_t mask;
  Grid(double hmin, double hmax, int64_t cap) {
    uint64_t t = 1024;
    while (t < (uint64_t)(2 * cap)) t <<= 1;
    mask = t - 1;
    for (double cs = hmin;; cs *= 2.0) {
      Level L;
      L.g = (int)std::floor(1.0 / cs);
      if (L.g < 1) L.g = 1;
      L.inv = (double)L.g;
      L.head.assign(t, -1);
      lv.push_back(std::move(L));
      next.emplace_back(cap, -1);
      if (cs >= hmax || lv.back().g <= 3) break;
    }
  }
  uint64_t bucket(int i, int j, int k) const {
    uint64_t h = (uint64_t)(uint32_t)i * 73856093ull ^ (uint64_t)(uint32_t)j * 19349663ull ^
                 (uint64_t)(uint32_t)k * 83492791ull;
    h ^= h >> 17;
    h *= 0xED5AD4BBull;
    h ^= h >> 11;
    return h & mask;
  }
  void insert(int32_t id, const double* x) {
    for (size_t l = 0; l < lv.size(); ++l) {
      Level& L = lv[l];
      int i = (int)(x[0] * L.inv) % L.g, j = (int)(x[1] * L.inv) % L.g, k = (int)(x[2] * L.inv) % L.g;
      uint64_t b = bucket(i, j, k);
      next[l][id] = L.head[b];
      L.head[b] = id;
    }
  }
  // true if some stored node lies strictly closer than rad to x
  bool occupied(const double* x, double rad, const double* pos) const {
    size_t l = 0;
    while (l + 1 < lv.size() && 1.0 / lv[l].inv < rad) ++l;
    const Level& L = lv[l];
    int ci = (int)(x[0] * L.inv) % L.g, cj = (int)(x[1] * L.inv) % L.g, ck = (int)(x[2] * L.inv) % L.g;
    double r2 = rad * rad;
    int span = (1.0 / L.inv >= rad) ? 1 : (int)std::ceil(rad * L.inv);
    for (int a = -span; a <= span; ++a)
      for (int b = -span; b <= span; ++b)
        for (int c = -span; c <= span; ++c) {
          int i = ((ci + a) % L.g + L.g) % L.g, j = ((cj + b) % L.g + L.g) % L.g,
              k = ((ck + c) % L.g + L.g) % L.g;
          for (int32_t m = L.head[bucket(i, j, k)]; m >= 0; m = next[l][m]) {
            const double* y = pos + 3 * (int64_t)m;
            double dx = mi(x[0] - y[0]), dy = mi(x[1] - y[1]), dz = mi(x[2] - y[2]);
            if (dx * dx + dy * dy + dz * dz < r2) return true;
          }
        }
    return false;
  }
};

int fill(double r, const Spacing& h, double hb, uint64_t seed, int n_cand, int64_t cap, double* pos, double* nrm,
         int64_t* n_out, int64_t* nb_out) {
  Cell cell{r};
  Rng rng(seed);
  Grid grid(std::fmin(h.lo(), hb), h.hi(), cap);
  int64_t n = 0;
  auto h_at = [&](const double* x) { return h(cell.sdf(x)); };

  // random rotation: orthonormal frame from two random directions
  double R[3][3];
  {
    double a[3], b[3];
    rng.unit(a);
    do {
      rng.unit(b);
    } while (std::fabs(a[0] * b[0] + a[1] * b[1] + a[2] * b[2]) > 0.9);
    double d = a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
    for (int i = 0; i < 3; ++i) b[i] -= d * a[i];
    double nb = std::sqrt(b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
    for (int i = 0; i < 3; ++i) b[i] /= nb;
    double c[3] = {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
    for (int i = 0; i < 3; ++i) { R[i][0] = a[i]; R[i][1] = b[i]; R[i][2] = c[i]; }
  }
  if (r > 0.0) {
    int64_t ns = (int64_t)std::llround(4.0 * M_PI * r * r / (1.15 * hb * hb));
    if (ns < 1) ns = 1;
    const double ga = M_PI * (3.0 - std::sqrt(5.0));
    for (int64_t i = 0; i < ns; ++i) {
      double z = 1.0 - (2.0 * i + 1.0) / (double)ns, rho = std::sqrt(std::fmax(0.0, 1.0 - z * z));
      double ph = ga * (double)i;
      double u0[3] = {rho * std::cos(ph), rho * std::sin(ph), z}, u[3];
      for (int a = 0; a < 3; ++a) u[a] = R[a][0] * u0[0] + R[a][1] * u0[1] + R[a][2] * u0[2];
      double x[3] = {0.5 + r * u[0], 0.5 + r * u[1], 0.5 + r * u[2]};
      if (x[0] < 0.0 || x[0] >= 1.0 || x[1] < 0.0 || x[1] >= 1.0 || x[2] < 0.0 || x[2] >= 1.0) continue;
      // where the grain meets an image of itself (r > 1/2) the two surfaces
      // are sampled independently up to their intersection; keep one of any
      // two points closer than half the surface spacing
      if (grid.occupied(x, 0.5 * hb, pos)) continue;
      if (n >= cap) { *n_out = n; return 1; }
      for (int a = 0; a < 3; ++a) { pos[3 * n + a] = x[a]; nrm[3 * n + a] = u[a]; }
      grid.insert((int32_t)n, x);
      ++n;
    }
  }
  *nb_out = n;
  int64_t head = 0;
  if (n == 0) {  // no grain: seed the front with one random fluid point
    double x[3] = {rng.uniform(), rng.uniform(), rng.uniform()};
    for (int a = 0; a < 3; ++a) { pos[a] = x[a]; nrm[a] = 0.0; }
    grid.insert(0, x);
    n = 1;
  }
  while (head < n) {
    const double* xd = pos + 3 * head;
    double hd = h_at(xd);
    for (int c = 0; c < n_cand; ++c) {
      double u[3];
      rng.unit(u);
      double x[3] = {wrap(xd[0] + hd * u[0]), wrap(xd[1] + hd * u[1]), wrap(xd[2] + hd * u[2])};
      double d = cell.sdf(x);
      if (!(d > 0.0)) continue;
      double hc = h(d);
      // no fluid node closer to the wall than half its spacing: where clipped
      // surface lattices meet at the cell faces (r > 1/2) the surface sampling
      // can leave room for one
      if (d < 0.5 * hc) continue;
      // exclusion radius: the smaller of the two target spacings, so that a
      // candidate spawned outward (where h grows) is not rejected by its parent
      if (grid.occupied(x, 0.999 * std::fmin(hc, hd), pos)) continue;
      if (n >= cap) { *n_out = n; return 1; }
      for (int a = 0; a < 3; ++a) { pos[3 * n + a] = x[a]; nrm[3 * n + a] = 0.0; }
      grid.insert((int32_t)n, x);
      ++n;
    }
    ++head;
  }
  *n_out = n;
  return 0;
}

}  // namespace

extern "C" {

// Returns 0 on success, 1 if cap was too small (n_out then holds the count
// reached), 2 on bad arguments.  pos and nrm are [cap][3]; boundary nodes come
// first (nb_out of them, with normals), interior nodes after them.
int nc_fill(double r, double h0, double slope, double hmax, double hb, uint64_t seed, int n_cand,
            int64_t cap, double* pos, double* nrm, int64_t* n_out, int64_t* nb_out) {
  if (!(r >= 0.0 && r < 0.70710678) || !(h0 > 0.0) || !(hmax >= h0) || !(hb > 0.0) || slope < 0.0 ||
      n_cand < 1 || cap < 1)
    return 2;
  return fill(r, Spacing{0, h0, slope, hmax, 1.0}, hb, seed, n_cand, cap, pos, nrm, n_out, nb_out);
}

// The same fill with the Gaussian refinement of Sec. 2.4.
int nc_fill_gauss(double r, double hmin, double hmax, double eps, double hb, uint64_t seed, int n_cand,
                  int64_t cap, double* pos, double* nrm, int64_t* n_out, int64_t* nb_out) {
  if (!(r >= 0.0 && r < 0.70710678) || !(hmin > 0.0) || !(hmax >= hmin) || !(eps > 0.0) || !(hb > 0.0) ||
      n_cand < 1 || cap < 1)
    return 2;
  return fill(r, Spacing{1, hmin, hmax, eps, std::sqrt(3.0) / 2.0 - r}, hb, seed, n_cand, cap, pos, nrm, n_out,
              nb_out);
}
}
