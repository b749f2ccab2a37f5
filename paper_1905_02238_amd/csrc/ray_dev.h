// ray_dev.h -- wave-cooperative ray traversal on occupancy grids (gfx950).
//
// The paper takes the beam's cells, in ascending distance, as the input of the
// MI algorithms (Sec. 2.2, Sec. 3.1) and projects 3D beams onto equal virtual
// cells before run-length encoding them (Sec. 4).  Both walks are done by one
// wave per ray.
//
// 2D grid walk.  The faces crossed along x sit at t_x(i) = (f_x(i) - p_x) *
// (1/d_x), with f_x(i) = f_x(0) + s_x i an integer, two roundings and no FMA,
// and likewise along y; the walk visits cells in the order of the merged,
// strictly increasing event times, an exact x/y tie being one diagonal step.
// Each lane produces event times independently, and an event's place in the
// merged order is its own index plus the number of events of the other axis
// strictly before it (count_below), minus the ties strictly before it.
// This reproduces, bit for bit, the sequential walk that steps whichever face
// is nearer: same event values, same order, same cells.
#pragma once
#include "fsmi_dev.h"

namespace fsmi {

// The distance along the ray to face i of one axis: ((f0 + s i) - p) * inv,
// two separately rounded operations after the exact integer face, so every
// evaluation of the same face gives the same bits.
struct FaceTimes {
  double f0, p, inv;
  int s;
  FSMI_DEV double operator()(int i) const {
#pragma clang fp contract(off)
    return ((f0 + (double)(s * i)) - p) * inv;
  }
};

// Count of faces i in [0, N) with A(i) < key, where A(i) is non-decreasing and
// A(i) ~ A(0) + i / rate (rate = |d| of that axis).  The spacing gives the
// count to within rounding; the two loops then move it to the exact boundary
// with the true comparisons, so the result is exact for any input (usually
// after one or two evaluations).  When the count c is below N, *at receives
// A(c), the first face time at or after key (every path evaluates it).
FSMI_DEV int count_below(const FaceTimes& A, int N, double key, double rate, double* at) {
  if (N <= 0) return 0;
  const double e = (key - A(0)) * rate;
  int c = !(e > 0.0) ? 0 : (e >= (double)N ? N : (int)ceil(e));
  bool down = false;
  while (c > 0) {
    const double v = A(c - 1);
    if (v < key) break;
    --c;
    *at = v;
    down = true;
  }
  if (!down) {
    while (c < N) {
      const double v = A(c);
      if (v >= key) {
        *at = v;
        break;
      }
      ++c;
    }
  }
  return c;
}

// Per-axis capacity for max range R: at most floor(R) + 3 faces per axis.
__host__ __device__ inline int dda2d_axis_cap(double R) { return (int)floor(R) + 3; }
// Capacity of per-event arrays: K events <= R(|dx| + |dy|) + 6 <= sqrt(2) R + 6.
__host__ __device__ inline int dda2d_event_cap(double R) {
  return (int)floor(1.4142135623730951 * R) + 8;
}

struct Dda2dResult {
  int n;          // number of cells (-1: origin outside / bad direction, -2: capacity)
  int skip0;      // 1 if the origin cell has zero length and is not listed
  int64_t cell0;  // origin cell
  double lend;    // l_{n+1}
};

// The walk.  tx, ty: LDS [capa] each; tie: LDS [capa + 1].  For every event the
// functor emit(r, t, c) receives its merged rank r, its time t and the cell the
// ray enters (linear index, or -1 outside the map).  Cell q of the result
// (q = 0..n-1) is the origin cell if q + skip0 == 0, else the cell entered at
// event r = q + skip0 - 1, with entry max(t, +0).  Events at ranks past the
// first exit are emitted too and must be ignored by the caller (ranks < ecap).
template <class Emit>
FSMI_DEV Dda2dResult dda2d_wave(int64_t X, int64_t Y, double px, double py, double dx, double dy,
                                double R, int capa, int ecap, int* tiep, Emit emit, int lane) {
#pragma clang fp contract(off)
  Dda2dResult res;
  res.n = -1;
  res.skip0 = 0;
  res.cell0 = 0;
  res.lend = 0.0;
  if (!(px >= 0.0 && px < (double)X && py >= 0.0 && py < (double)Y)) return res;
  if (dx == 0.0 && dy == 0.0) return res;
  // The map has fewer than 2^31 cells (checked at the boundary), so cell
  // coordinates, the one-past-the-edge ones included, and indices fit int32.
  const int Xi = (int)X, Yi = (int)Y;
  const int cx0 = (int)floor(px), cy0 = (int)floor(py);
  res.cell0 = cx0 + (int64_t)Xi * cy0;
  const int sx = dx > 0.0 ? 1 : (dx < 0.0 ? -1 : 0);
  const int sy = dy > 0.0 ? 1 : (dy < 0.0 ? -1 : 0);
  const double fx0 = sx > 0 ? (double)(cx0 + 1) : (double)cx0;
  const double fy0 = sy > 0 ? (double)(cy0 + 1) : (double)cy0;
  const double ix = sx ? 1.0 / dx : 0.0;
  const double iy = sy ? 1.0 / dy : 0.0;
  const double adx = fabs(dx), ady = fabs(dy);   // events per unit of t, per axis
  const FaceTimes tx{fx0, px, ix, sx}, ty{fy0, py, iy, sy};   // face times, recomputed on use
  const int64_t ex = sx > 0 ? X - 1 - cx0 : cx0;   // x event index that leaves the map
  const int64_t ey = sy > 0 ? Y - 1 - cy0 : cy0;
  int nx = 0, ny = 0;
  if (sx) nx = (int)min<int64_t>(ex, (int64_t)floor(R * fabs(dx)) + 2) + 1;
  if (sy) ny = (int)min<int64_t>(ey, (int64_t)floor(R * fabs(dy)) + 2) + 1;
  if (nx > capa || ny > capa || nx + ny + 1 > ecap) {
    res.n = -2;
    return res;
  }
  // events before R (the times increase, so they form a prefix); the same
  // count in every lane
  double unused;
  const int Nx = count_below(tx, nx, R, adx, &unused);
  const int Ny = count_below(ty, ny, R, ady, &unused);
  // the first event decides whether the origin cell has zero length
  double t0 = 1.0 / 0.0;
  if (Nx > 0) t0 = tx(0);
  if (Ny > 0 && ty(0) < t0) t0 = ty(0);
  int first_out = 0x7fffffff;   // rank of the first event that leaves the map
  double t_out = 0.0;
  // x events, a chunk of 64 at a time: the y events before each, its tie (an
  // equal y event time: one diagonal step), the exclusive prefix count of ties
  // (kept for the y events), its rank, and the cell it enters
  int carry = 0;
  for (int base = 0; base < Nx; base += kWave) {
    const int i = base + lane;
    int tie = 0, c = 0;
    double t = 0.0;
    if (i < Nx) {
      t = tx(i);
      double at = 0.0;
      c = count_below(ty, Ny, t, ady, &at);
      tie = (c < Ny && at == t) ? 1 : 0;
    }
    const int inc = wave_scan_incl<OpAdd>(tie);
    if (i < Nx) {
      const int before = carry + inc - tie;
      tiep[i] = before;
      const int r = i + c - before;
      const int cx = cx0 + sx * (i + 1);
      const int cy = cy0 + sy * (c + tie);
      const bool in = cx >= 0 && cx < Xi && cy >= 0 && cy < Yi;
      if (!in && r < first_out) first_out = r, t_out = t;
      emit(r, t, in ? cx + Xi * cy : -1);
    }
    carry += wave_last(inc);
  }
  if (lane == 0) tiep[Nx] = carry;
  wave_sync();
  const int K = Nx + Ny - carry;
  res.skip0 = (K >= 1 && !(t0 > 0.0)) ? 1 : 0;
  // y events that do not tie with an x event
  for (int m = lane; m < Ny; m += kWave) {
    const double t = ty(m);
    double at = 0.0;
    const int c = count_below(tx, Nx, t, adx, &at);
    if (c < Nx && at == t) continue;
    const int r = m + c - tiep[c];
    const int cy = cy0 + sy * (m + 1);
    const int cx = cx0 + sx * c;
    const bool in = cx >= 0 && cx < Xi && cy >= 0 && cy < Yi;
    if (!in && r < first_out) first_out = r, t_out = t;
    emit(r, t, in ? cx + Xi * cy : -1);
  }
  const int mine = first_out;
  first_out = wave_min(first_out);
  int ncand;
  if (first_out < K) {
    ncand = first_out + 1;   // cells 0..first_out; the walk ends at that event
    const uint64_t who = __ballot(mine == first_out);
    const int src = (int)__builtin_ctzll(who);
    int2 tb = *reinterpret_cast<int2*>(&t_out);
    tb.x = __builtin_amdgcn_readlane(tb.x, src);
    tb.y = __builtin_amdgcn_readlane(tb.y, src);
    const double te = *reinterpret_cast<double*>(&tb);
    res.lend = te > 0.0 ? te : 0.0;
  } else {
    ncand = K + 1;
    res.lend = R;
  }
  res.n = ncand - res.skip0;
  wave_sync();
  return res;
}

// ---------------------------------------------------------------------------
// 3D virtual cells of width w: sample i = 1..floor(R/w) at the midpoint
// p + t_i d, t_i = (i - 1/2) w, per axis without FMA; the beam ends at the
// first midpoint outside the map.  Writes o (and the cell index if asked) to
// LDS, returns n.
// ---------------------------------------------------------------------------
FSMI_DEV int virtual3d_wave(const float* __restrict__ map, int64_t X, int64_t Y, int64_t Z,
                            const double* p, const double* d, double R, double w, int cap,
                            float* so, int* scell, int lane, bool* origin_ok) {
#pragma clang fp contract(off)
  *origin_ok = p[0] >= 0.0 && p[0] < (double)X && p[1] >= 0.0 && p[1] < (double)Y &&
               p[2] >= 0.0 && p[2] < (double)Z;
  if (!*origin_ok) return 0;
  const int64_t nmax = (int64_t)floor(R / w);
  int n = (int)min<int64_t>(nmax, (int64_t)cap);
  int end = n;
  // pass 1: voxel indices (in o's slots) and the first sample outside the map
  int* sidx = reinterpret_cast<int*>(so);
  for (int base = 0; base < n; base += kWave) {
    const int i = base + lane + 1;
    bool in = false;
    int64_t idx = 0;
    if (i <= n) {
      const double t = ((double)i - 0.5) * w;
      const double qx = p[0] + t * d[0];
      const double qy = p[1] + t * d[1];
      const double qz = p[2] + t * d[2];
      const double vx = floor(qx), vy = floor(qy), vz = floor(qz);
      in = vx >= 0.0 && vx < (double)X && vy >= 0.0 && vy < (double)Y && vz >= 0.0 && vz < (double)Z;
      if (in) idx = (int64_t)vx + X * ((int64_t)vy + Y * (int64_t)vz);
    }
    const uint64_t outm = __ballot(i <= n && !in);
    if (i <= n && in) {
      sidx[i - 1] = (int)idx;
      if (scell) scell[i - 1] = (int)idx;
    }
    if (outm) {
      end = base + __builtin_ctzll(outm);
      break;
    }
  }
  wave_sync();
  // pass 2: the occupancies of samples 0 .. end-1 (all inside the map), four
  // loads in flight per lane
  for (int b0 = 0; b0 < end; b0 += 4 * kWave) {
    int c[4];
    float o[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = b0 + u * kWave + lane;
      c[u] = i < end ? sidx[i] : 0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) o[u] = map[c[u]];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = b0 + u * kWave + lane;
      if (i < end) so[i] = o[u];
    }
  }
  wave_sync();
  return end;
}

// Maximal runs of bit-identical o in so[0..n): run values, run lengths and start
// indices (Eq. occup_rle).  Returns the number of runs.
FSMI_DEV int runs_wave(const float* so, int n, float* ro, int* rl, int* rs, int lane) {
  int carry = 0;
  for (int base = 0; base < n; base += kWave) {
    const int i = base + lane;
    int head = 0;
    if (i < n) head = (i == 0 || __float_as_uint(so[i]) != __float_as_uint(so[i - 1])) ? 1 : 0;
    const int inc = wave_scan_incl<OpAdd>(head);
    if (head) {
      const int r = carry + inc - 1;
      ro[r] = so[i];
      rs[r] = i;
    }
    carry += wave_last(inc);
  }
  wave_sync();
  const int nr = carry;
  for (int r = lane; r < nr; r += kWave) rl[r] = (r + 1 < nr ? rs[r + 1] : n) - rs[r];
  wave_sync();
  return nr;
}

}  // namespace fsmi
