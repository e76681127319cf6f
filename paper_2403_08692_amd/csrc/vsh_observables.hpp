// vsh_observables.hpp -- per-event observables of Sec. 3.1 (validation,
// exact thrust, Durham y23/y34, C-parameter, hemisphere masses and
// broadenings) and the histogram binning, one thread per event.
#pragma once

#include "vsh_kernels.hpp"

namespace vsh {

// ---------------------------------------------------------------------------
// Observables, one thread per event (Sec. 3.1).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double len3(double x, double y, double z) {
  return sqrt(x * x + y * y + z * z);
}

// exact thrust by the plane enumeration: pairs (i<j) span candidate planes,
// every other momentum sits on one side; i and j take all four sign choices
__device__ __forceinline__ double thrust_of(const Records& r, uint64_t e, int n, double sum, double& ax,
                            double& ay, double& az) {
  double best = -1.0, bx = 0.0, by = 0.0, bz = 1.0;
  if (n < 3) {
    for (int m = 0; m < (1 << n); ++m) {
      double vx = 0.0, vy = 0.0, vz = 0.0;
      for (int a = 0; a < n; ++a) {
        const double sg = (m >> a & 1) ? -1.0 : 1.0;
        const uint64_t o = (uint64_t)a * r.stride + e;
        vx += sg * r.x[o];
        vy += sg * r.y[o];
        vz += sg * r.z[o];
      }
      const double m2 = vx * vx + vy * vy + vz * vz;
      if (m2 > best) { best = m2; bx = vx; by = vy; bz = vz; }
    }
  } else {
    for (int i = 0; i < n; ++i) {
      const uint64_t oi = (uint64_t)i * r.stride + e;
      const double xi = r.x[oi], yi = r.y[oi], zi = r.z[oi];
      for (int j = i + 1; j < n; ++j) {
        const uint64_t oj = (uint64_t)j * r.stride + e;
        const double xj = r.x[oj], yj = r.y[oj], zj = r.z[oj];
        const double nx = yi * zj - zi * yj, ny = zi * xj - xi * zj, nz = xi * yj - yi * xj;
        double vx = 0.0, vy = 0.0, vz = 0.0;
        for (int k = 0; k < n; ++k) {
          if (k == i || k == j) continue;
          const uint64_t ok = (uint64_t)k * r.stride + e;
          const double xk = r.x[ok], yk = r.y[ok], zk = r.z[ok];
          const double d = xk * nx + yk * ny + zk * nz;
          if (d > 0.0) { vx += xk; vy += yk; vz += zk; }
          else { vx -= xk; vy -= yk; vz -= zk; }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double si = (c < 2) ? 1.0 : -1.0, sj = (c & 1) ? -1.0 : 1.0;
          const double wx = vx + si * xi + sj * xj, wy = vy + si * yi + sj * yj,
                       wz = vz + si * zi + sj * zj;
          const double m2 = wx * wx + wy * wy + wz * wz;
          if (m2 > best) { best = m2; bx = wx; by = wy; bz = wz; }
        }
      }
    }
  }
  const double l = sqrt(best);
  if (l > 0.0) { ax = bx / l; ay = by / l; az = bz / l; }
  else { ax = 0.0; ay = 0.0; az = 1.0; }
  return sum > 0.0 ? l / sum : 0.0;
}

// Durham clustering, E-scheme; y_ab = min(E_a,E_b)^2 |u_a - u_b|^2 / s
__device__ __forceinline__ void durham_of(const Records& r, const Scratch& sc, uint64_t e, uint64_t slot, int n, double sh,
                          double& y23, double& y34) {
  for (int a = 0; a < n; ++a) {
    const uint64_t o = (uint64_t)a * r.stride + e;
    const uint64_t q = (uint64_t)a * sc.stride + slot;
    sc.jE[q] = r.E[o];
    sc.jx[q] = r.x[o];
    sc.jy[q] = r.y[o];
    sc.jz[q] = r.z[o];
  }
  y23 = 0.0;
  y34 = 0.0;
  int m = n;
  while (m > 2) {
    double ymin = 0.0;
    int ba = -1, bb = -1;
    for (int a = 0; a < m; ++a) {
      const uint64_t qa = (uint64_t)a * sc.stride + slot;
      const double ea = sc.jE[qa], xa = sc.jx[qa], ya = sc.jy[qa], za = sc.jz[qa];
      const double la = len3(xa, ya, za);
      for (int b = a + 1; b < m; ++b) {
        const uint64_t qb = (uint64_t)b * sc.stride + slot;
        const double eb = sc.jE[qb], xb = sc.jx[qb], yb = sc.jy[qb], zb = sc.jz[qb];
        const double lb = len3(xb, yb, zb);
        const double dx = xa / la - xb / lb, dy = ya / la - yb / lb, dz = za / la - zb / lb;
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        const double em = ea < eb ? ea : eb;
        const double yv = em * em * d2 / sh;
        if (ba < 0 || yv < ymin) { ymin = yv; ba = a; bb = b; }
      }
    }
    if (m == 4) y34 = ymin;
    if (m == 3) y23 = ymin;
    const uint64_t qa = (uint64_t)ba * sc.stride + slot;
    const uint64_t qb = (uint64_t)bb * sc.stride + slot;
    sc.jE[qa] += sc.jE[qb];
    sc.jx[qa] += sc.jx[qb];
    sc.jy[qa] += sc.jy[qb];
    sc.jz[qa] += sc.jz[qb];
    for (int a = bb; a + 1 < m; ++a) {
      const uint64_t q0 = (uint64_t)a * sc.stride + slot, q1 = q0 + sc.stride;
      sc.jE[q0] = sc.jE[q1];
      sc.jx[q0] = sc.jx[q1];
      sc.jy[q0] = sc.jy[q1];
      sc.jz[q0] = sc.jz[q1];
    }
    --m;
  }
}

__device__ __forceinline__ int bin_of(double x, double lo, double hi) {
  if (x != x) return kNBins + 1;
  if (x < lo) return 0;
  if (x >= hi) return kNBins + 1;
  int b = 1 + (int)((x - lo) / (hi - lo) * kNBins);
  return b > kNBins ? kNBins : b;
}

struct ObsOut {
  double v[7];  // y23, y34, tau, C, rho_H, B_T, B_W
  int status;
};

// Validate the event (finite; four-momentum conserved to 1e-10 sqrt(s) per
// component; every parton massless to 1e-10 s) and, if it passes, compute
// its observables.
__device__ __forceinline__ ObsOut event_observables(const Records& r, const Scratch& sc, uint64_t e,
                                                    uint64_t slot, int np, double ecm, int status) {
  ObsOut o;
  for (int h = 0; h < 7; ++h) o.v[h] = 0.0;
  const double sh = ecm * ecm;
  if (status == kDone) {
    double tE = 0.0, tx = 0.0, ty = 0.0, tz = 0.0;
    bool finite = true, massless = true;
    for (int a = 0; a < np; ++a) {
      const P4 p = r.load(a, e);
      finite = finite && isfinite(p.e) && isfinite(p.x) && isfinite(p.y) && isfinite(p.z);
      tE += p.e;
      tx += p.x;
      ty += p.y;
      tz += p.z;
      massless = massless && fabs(mdot(p, p)) <= 1e-10 * sh;
    }
    const double tol = 1e-10 * ecm;
    if (!finite) status = kNonFinite;
    else if (fabs(tE - ecm) > tol || fabs(tx) > tol || fabs(ty) > tol || fabs(tz) > tol || !massless)
      status = kConservation;
  }
  o.status = status;
  if (status != kDone) return o;
  double sum = 0.0;
  for (int a = 0; a < np; ++a) {
    const uint64_t q = (uint64_t)a * r.stride + e;
    sum += len3(r.x[q], r.y[q], r.z[q]);
  }
  double ax, ay, az;
  const double T = thrust_of(r, e, np, sum, ax, ay, az);
  durham_of(r, sc, e, slot, np, sh, o.v[0], o.v[1]);
  const double tau = 1.0 - T;
  o.v[2] = tau > 0.0 ? tau : 0.0;
  double dbl = 0.0;
  for (int a = 0; a < np; ++a) {
    const uint64_t qa = (uint64_t)a * r.stride + e;
    const double xa = r.x[qa], ya = r.y[qa], za = r.z[qa], la = len3(xa, ya, za);
    for (int b = 0; b < np; ++b) {
      const uint64_t qb = (uint64_t)b * r.stride + e;
      const double xb = r.x[qb], yb = r.y[qb], zb = r.z[qb], lb = len3(xb, yb, zb);
      const double d = xa * xb + ya * yb + za * zb;
      dbl += d * d / (la * lb);
    }
  }
  const double cpar = 1.5 * (sum * sum - dbl) / (sum * sum);
  o.v[3] = cpar > 0.0 ? cpar : 0.0;
  P4 hp{0, 0, 0, 0}, hm{0, 0, 0, 0};
  double bp = 0.0, bm = 0.0;
  for (int a = 0; a < np; ++a) {
    const P4 q = r.load(a, e);
    const double d = q.x * ax + q.y * ay + q.z * az;
    const double kt = len3(q.y * az - q.z * ay, q.z * ax - q.x * az, q.x * ay - q.y * ax);
    if (d >= 0.0) {
      hp.e += q.e; hp.x += q.x; hp.y += q.y; hp.z += q.z; bp += kt;
    } else {
      hm.e += q.e; hm.x += q.x; hm.y += q.y; hm.z += q.z; bm += kt;
    }
  }
  const double mp = mdot(hp, hp), mm = mdot(hm, hm);
  const double rho = (mp > mm ? mp : mm) / sh;
  o.v[4] = rho > 0.0 ? rho : 0.0;
  bp /= 2.0 * sum;
  bm /= 2.0 * sum;
  o.v[5] = bp + bm;
  o.v[6] = bp > bm ? bp : bm;
  return o;
}

__device__ __forceinline__ double hist_lo(int h) {
  return h < 2 ? -4.3 : (h == 7 ? -1.0 : 0.0);
}
__device__ __forceinline__ double hist_hi(int h) {
  return h < 2 ? -0.3 : (h == 3 ? 1.0 : (h == 6 ? 0.35 : (h == 7 ? 1.0 : 0.5)));
}

// Fill one event into an LDS histogram set [kNObs][kNHCol][3].
__device__ __forceinline__ void hist_fill_lds(double* lh, const ObsOut& o, double w, double cos_theta) {
  double vals[kNObs];
  vals[0] = o.v[0] > 0.0 ? log10(o.v[0]) : -INFINITY;
  vals[1] = o.v[1] > 0.0 ? log10(o.v[1]) : -INFINITY;
  for (int h = 2; h < 7; ++h) vals[h] = o.v[h];
  vals[7] = cos_theta;
#pragma unroll
  for (int h = 0; h < kNObs; ++h) {
    const int b = bin_of(vals[h], hist_lo(h), hist_hi(h));
    double* cell = &lh[3 * (kNHCol * h + b)];
    atomicAdd(&cell[0], w);
    atomicAdd(&cell[1], w * w);
    atomicAdd(&cell[2], 1.0);
  }
}

}  // namespace vsh
