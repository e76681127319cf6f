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

// ---------------------------------------------------------------------------
// Scratch-based observables.  The event's partons are first copied to a
// per-thread scratch laid out [slot][thread] (lanes of a wave hold events of
// equal size after the sort by parton count, so every pass below reads
// consecutive addresses), then:
//   validation, thrust (plane enumeration, first maximum), hemispheres,
//   C from the momentum tensor M_ab = sum_i p_i^a p_i^b / |p_i|:
//     sum_ij (p_i.p_j)^2/(|p_i||p_j|) = sum_ab M_ab^2,
//   and Durham with forward nearest neighbours: for each jet a the smallest
//   y(a, b) over later jets b (first b on ties); the global minimum over a
//   (first a on ties) is then the first minimum of the pair scan in (a, b)
//   order.  After a merge of (i, j), i < j, only jets whose neighbour was i
//   or j need a rescan; earlier jets compare against the new i.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double durham_y(const Scratch& w, uint64_t qa, uint64_t qb, double inv_s) {
  const double dx = w.ux[qa] - w.ux[qb], dy = w.uy[qa] - w.uy[qb], dz = w.uz[qa] - w.uz[qb];
  const double d2 = (dx * dx + dy * dy) + dz * dz;
  const double ea = w.E[qa], eb = w.E[qb];
  const double em = ea < eb ? ea : eb;
  return em * em * d2 * inv_s;
}

__device__ __forceinline__ void set_unit(const Scratch& w, uint64_t q) {
  const double l = len3(w.x[q], w.y[q], w.z[q]);
  w.ux[q] = w.x[q] / l;
  w.uy[q] = w.y[q] / l;
  w.uz[q] = w.z[q] / l;
}

// forward nearest neighbour of alive jet a among alive jets b > a
__device__ __forceinline__ void forward_nn(const Scratch& w, uint64_t t, int a, int n, double inv_s) {
  const uint64_t qa = (uint64_t)a * w.stride + t;
  double best = 0.0;
  int bb = -1;
  for (int b = a + 1; b < n; ++b) {
    if (w.dead[(uint64_t)b * w.stride + t]) continue;
    const double y = durham_y(w, qa, (uint64_t)b * w.stride + t, inv_s);
    if (bb < 0 || y < best) {
      best = y;
      bb = b;
    }
  }
  w.nn[qa] = bb < 0 ? (uint16_t)0xFFFF : (uint16_t)bb;
  w.dn[qa] = best;
}

__device__ void durham_nn(const Scratch& w, uint64_t t, int n, double sh, double& y23, double& y34) {
  const double inv_s = 1.0 / sh;
  y23 = 0.0;
  y34 = 0.0;
  if (n < 3) return;
  for (int a = 0; a < n; ++a) {
    w.dead[(uint64_t)a * w.stride + t] = 0;
    set_unit(w, (uint64_t)a * w.stride + t);
  }
  for (int a = 0; a < n; ++a) forward_nn(w, t, a, n, inv_s);
  int m = n;
  while (m > 2) {
    int ia = -1;
    double ymin = 0.0;
    for (int a = 0; a < n; ++a) {
      const uint64_t qa = (uint64_t)a * w.stride + t;
      if (w.dead[qa] || w.nn[qa] == 0xFFFF) continue;
      const double d = w.dn[qa];
      if (ia < 0 || d < ymin) {
        ymin = d;
        ia = a;
      }
    }
    const int i = ia, j = w.nn[(uint64_t)ia * w.stride + t];
    if (m == 4) y34 = ymin;
    if (m == 3) y23 = ymin;
    const uint64_t qi = (uint64_t)i * w.stride + t, qj = (uint64_t)j * w.stride + t;
    w.E[qi] += w.E[qj];
    w.x[qi] += w.x[qj];
    w.y[qi] += w.y[qj];
    w.z[qi] += w.z[qj];
    set_unit(w, qi);
    w.dead[qj] = 1;
    --m;
    if (m <= 2) break;
    forward_nn(w, t, i, n, inv_s);
    for (int a = 0; a < n; ++a) {
      const uint64_t qa = (uint64_t)a * w.stride + t;
      if (w.dead[qa] || a == i) continue;
      const int na = w.nn[qa];
      if (na == i || na == j) {
        forward_nn(w, t, a, n, inv_s);
      } else if (a < i) {
        const double y = durham_y(w, qa, qi, inv_s);
        if (na == 0xFFFF || y < w.dn[qa] || (y == w.dn[qa] && i < na)) {
          w.nn[qa] = (uint16_t)i;
          w.dn[qa] = y;
        }
      }
    }
  }
}

// Squared mass shell of parton a of event e of r: zero unless the request
// gives quark masses (the kMassive instantiations of the passes).
template <bool kMassive>
__device__ __forceinline__ double shell2(const EventInputs& in, const Records& r, int a, uint64_t e) {
  if constexpr (!kMassive) {
    return 0.0;
  } else {
    const double m = quark_mass(in.qm, r.pid[(uint64_t)a * r.stride + e]);
    return m * m;
  }
}

// Observables of one event (e of r) whose n partons are in scratch column t.
template <bool kMassive>
__device__ __forceinline__ ObsOut scratch_observables(const Scratch& w, uint64_t t, int np, double ecm,
                                                      int status, const EventInputs& in, const Records& r,
                                                      uint64_t e) {
  ObsOut o;
  for (int h = 0; h < 7; ++h) o.v[h] = 0.0;
  const double sh = ecm * ecm;
  if (status == kDone) {
    double tE = 0.0, tx = 0.0, ty = 0.0, tz = 0.0;
    bool finite = true, on_shell = true;
    for (int a = 0; a < np; ++a) {
      const uint64_t q = (uint64_t)a * w.stride + t;
      const P4 p{w.E[q], w.x[q], w.y[q], w.z[q]};
      finite = finite && isfinite(p.e) && isfinite(p.x) && isfinite(p.y) && isfinite(p.z);
      tE += p.e;
      tx += p.x;
      ty += p.y;
      tz += p.z;
      on_shell = on_shell && fabs(mdot(p, p) - shell2<kMassive>(in, r, a, e)) <= 1e-10 * sh;
    }
    const double tol = 1e-10 * ecm;
    if (!finite) status = kNonFinite;
    else if (fabs(tE - ecm) > tol || fabs(tx) > tol || fabs(ty) > tol || fabs(tz) > tol || !on_shell)
      status = kConservation;
  }
  o.status = status;
  if (status != kDone) return o;
  // sum |p| and the momentum tensor
  double sum = 0.0, mxx = 0.0, myy = 0.0, mzz = 0.0, mxy = 0.0, mxz = 0.0, myz = 0.0;
  for (int a = 0; a < np; ++a) {
    const uint64_t q = (uint64_t)a * w.stride + t;
    const double x = w.x[q], y = w.y[q], z = w.z[q];
    const double l = len3(x, y, z);
    sum += l;
    const double il = 1.0 / l;
    mxx += x * x * il;
    myy += y * y * il;
    mzz += z * z * il;
    mxy += x * y * il;
    mxz += x * z * il;
    myz += y * z * il;
  }
  // thrust
  double best = -1.0, bx = 0.0, by = 0.0, bz = 1.0;
  if (np < 3) {
    for (int mk = 0; mk < (1 << np); ++mk) {
      double vx = 0.0, vy = 0.0, vz = 0.0;
      for (int a = 0; a < np; ++a) {
        const double sg = (mk >> a & 1) ? -1.0 : 1.0;
        const uint64_t q = (uint64_t)a * w.stride + t;
        vx += sg * w.x[q];
        vy += sg * w.y[q];
        vz += sg * w.z[q];
      }
      const double m2 = vx * vx + vy * vy + vz * vz;
      if (m2 > best) { best = m2; bx = vx; by = vy; bz = vz; }
    }
  } else {
    for (int i = 0; i < np; ++i) {
      const uint64_t qi = (uint64_t)i * w.stride + t;
      const double xi = w.x[qi], yi = w.y[qi], zi = w.z[qi];
      for (int j = i + 1; j < np; ++j) {
        const uint64_t qj = (uint64_t)j * w.stride + t;
        const double xj = w.x[qj], yj = w.y[qj], zj = w.z[qj];
        const double nx = yi * zj - zi * yj, ny = zi * xj - xi * zj, nz = xi * yj - yi * xj;
        double vx = 0.0, vy = 0.0, vz = 0.0;
        for (int k = 0; k < np; ++k) {
          if (k == i || k == j) continue;
          const uint64_t qk = (uint64_t)k * w.stride + t;
          const double xk = w.x[qk], yk = w.y[qk], zk = w.z[qk];
          const double d = xk * nx + yk * ny + zk * nz;
          if (d > 0.0) { vx += xk; vy += yk; vz += zk; }
          else { vx -= xk; vy -= yk; vz -= zk; }
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const double si = (c < 2) ? 1.0 : -1.0, sj = (c & 1) ? -1.0 : 1.0;
          const double wx = vx + si * xi + sj * xj, wy = vy + si * yi + sj * yj, wz = vz + si * zi + sj * zj;
          const double m2 = wx * wx + wy * wy + wz * wz;
          if (m2 > best) { best = m2; bx = wx; by = wy; bz = wz; }
        }
      }
    }
  }
  const double lb = sqrt(best);
  double ax = 0.0, ay = 0.0, az = 1.0;
  if (lb > 0.0) { ax = bx / lb; ay = by / lb; az = bz / lb; }
  const double T = sum > 0.0 ? lb / sum : 0.0;
  const double tau = 1.0 - T;
  o.v[2] = tau > 0.0 ? tau : 0.0;
  const double m2s = mxx * mxx + myy * myy + mzz * mzz + 2.0 * (mxy * mxy + mxz * mxz + myz * myz);
  const double cpar = 1.5 * (sum * sum - m2s) / (sum * sum);
  o.v[3] = cpar > 0.0 ? cpar : 0.0;
  P4 hp{0, 0, 0, 0}, hm{0, 0, 0, 0};
  double bp = 0.0, bm = 0.0;
  for (int a = 0; a < np; ++a) {
    const uint64_t q = (uint64_t)a * w.stride + t;
    const P4 p{w.E[q], w.x[q], w.y[q], w.z[q]};
    const double d = p.x * ax + p.y * ay + p.z * az;
    const double kt = len3(p.y * az - p.z * ay, p.z * ax - p.x * az, p.x * ay - p.y * ax);
    if (d >= 0.0) { hp.e += p.e; hp.x += p.x; hp.y += p.y; hp.z += p.z; bp += kt; }
    else { hm.e += p.e; hm.x += p.x; hm.y += p.y; hm.z += p.z; bm += kt; }
  }
  const double mp = mdot(hp, hp), mm = mdot(hm, hm);
  const double rho = (mp > mm ? mp : mm) / sh;
  o.v[4] = rho > 0.0 ? rho : 0.0;
  bp /= 2.0 * sum;
  bm /= 2.0 * sum;
  o.v[5] = bp + bm;
  o.v[6] = bp > bm ? bp : bm;
  durham_nn(w, t, np, sh, o.v[0], o.v[1]);  // last: merges jets in the scratch
  return o;
}

// ---------------------------------------------------------------------------
// Register observables for events of at most M partons: the same quantities
// in the same scan orders, with the partons held in registers (loops fully
// unrolled over M slots, guarded by the parton count, which is uniform over
// most waves after the sort).  Durham scans every alive pair (a < b) in order
// and keeps the first minimum, the same merge the nearest-neighbour version
// picks; a merge adds jet b into jet a.
// ---------------------------------------------------------------------------
template <int M, bool kMassive>
__device__ __forceinline__ ObsOut reg_observables(const Records& r, uint64_t e, int np, int wmax, double ecm,
                                                  int status, const EventInputs& in) {
  ObsOut o;
#pragma unroll
  for (int h = 0; h < 7; ++h) o.v[h] = 0.0;
  double E[M], X[M], Y[M], Z[M];
#pragma unroll
  for (int a = 0; a < M; ++a) {
    E[a] = X[a] = Y[a] = Z[a] = 0.0;
    if (a >= wmax) continue;  // wmax: the wave's largest parton count (uniform)
    if (a < np) {
      const P4 p = r.load(a, e);
      E[a] = p.e;
      X[a] = p.x;
      Y[a] = p.y;
      Z[a] = p.z;
    }
  }
  const double sh = ecm * ecm;
  if (status == kDone) {
    double tE = 0.0, tx = 0.0, ty = 0.0, tz = 0.0;
    bool finite = true, on_shell = true;
#pragma unroll
    for (int a = 0; a < M; ++a) {
      if (a < np) {
        const P4 p{E[a], X[a], Y[a], Z[a]};
        finite = finite && isfinite(p.e) && isfinite(p.x) && isfinite(p.y) && isfinite(p.z);
        tE += p.e;
        tx += p.x;
        ty += p.y;
        tz += p.z;
        on_shell = on_shell && fabs(mdot(p, p) - shell2<kMassive>(in, r, a, e)) <= 1e-10 * sh;
      }
    }
    const double tol = 1e-10 * ecm;
    if (!finite) status = kNonFinite;
    else if (fabs(tE - ecm) > tol || fabs(tx) > tol || fabs(ty) > tol || fabs(tz) > tol || !on_shell)
      status = kConservation;
  }
  o.status = status;
  if (status != kDone) return o;
  // sum |p| and the momentum tensor
  double sum = 0.0, mxx = 0.0, myy = 0.0, mzz = 0.0, mxy = 0.0, mxz = 0.0, myz = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    if (a < np) {
      const double x = X[a], y = Y[a], z = Z[a];
      const double l = len3(x, y, z);
      sum += l;
      const double il = 1.0 / l;
      mxx += x * x * il;
      myy += y * y * il;
      mzz += z * z * il;
      mxy += x * y * il;
      mxz += x * z * il;
      myz += y * z * il;
    }
  }
  // thrust
  double best = -1.0, bx = 0.0, by = 0.0, bz = 1.0;
  if (np < 3) {
    for (int mk = 0; mk < (1 << np); ++mk) {
      double vx = 0.0, vy = 0.0, vz = 0.0;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        if (a < np) {
          const double sg = (mk >> a & 1) ? -1.0 : 1.0;
          vx += sg * X[a];
          vy += sg * Y[a];
          vz += sg * Z[a];
        }
      }
      const double m2 = vx * vx + vy * vy + vz * vz;
      if (m2 > best) { best = m2; bx = vx; by = vy; bz = vz; }
    }
  } else {
    // the outer index runs as a loop (its momentum picked out of the
    // registers), the inner ones unrolled over the M slots
#pragma unroll 1
    for (int i = 0; i + 1 < np; ++i) {
      double xi = 0.0, yi = 0.0, zi = 0.0;
#pragma unroll
      for (int a = 0; a < M; ++a)
        if (a == i) { xi = X[a]; yi = Y[a]; zi = Z[a]; }
#pragma unroll
      for (int j = 1; j < M; ++j) {
        if (j >= wmax) break;
        if (j > i && j < np) {
          const double nx = yi * Z[j] - zi * Y[j], ny = zi * X[j] - xi * Z[j], nz = xi * Y[j] - yi * X[j];
          double vx = 0.0, vy = 0.0, vz = 0.0;
#pragma unroll
          for (int k = 0; k < M; ++k) {
            if (k >= wmax) break;
            if (k != i && k != j && k < np) {
              const double d = X[k] * nx + Y[k] * ny + Z[k] * nz;
              if (d > 0.0) { vx += X[k]; vy += Y[k]; vz += Z[k]; }
              else { vx -= X[k]; vy -= Y[k]; vz -= Z[k]; }
            }
          }
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const double si = (c < 2) ? 1.0 : -1.0, sj = (c & 1) ? -1.0 : 1.0;
            const double wx = vx + si * xi + sj * X[j], wy = vy + si * yi + sj * Y[j], wz = vz + si * zi + sj * Z[j];
            const double m2 = wx * wx + wy * wy + wz * wz;
            if (m2 > best) { best = m2; bx = wx; by = wy; bz = wz; }
          }
        }
      }
    }
  }
  const double lb = sqrt(best);
  double ax = 0.0, ay = 0.0, az = 1.0;
  if (lb > 0.0) { ax = bx / lb; ay = by / lb; az = bz / lb; }
  const double T = sum > 0.0 ? lb / sum : 0.0;
  const double tau = 1.0 - T;
  o.v[2] = tau > 0.0 ? tau : 0.0;
  const double m2s = mxx * mxx + myy * myy + mzz * mzz + 2.0 * (mxy * mxy + mxz * mxz + myz * myz);
  const double cpar = 1.5 * (sum * sum - m2s) / (sum * sum);
  o.v[3] = cpar > 0.0 ? cpar : 0.0;
  P4 hp{0, 0, 0, 0}, hm{0, 0, 0, 0};
  double bp = 0.0, bm = 0.0;
#pragma unroll
  for (int a = 0; a < M; ++a) {
    if (a < np) {
      const P4 p{E[a], X[a], Y[a], Z[a]};
      const double d = p.x * ax + p.y * ay + p.z * az;
      const double kt = len3(p.y * az - p.z * ay, p.z * ax - p.x * az, p.x * ay - p.y * ax);
      if (d >= 0.0) { hp.e += p.e; hp.x += p.x; hp.y += p.y; hp.z += p.z; bp += kt; }
      else { hm.e += p.e; hm.x += p.x; hm.y += p.y; hm.z += p.z; bm += kt; }
    }
  }
  const double mp = mdot(hp, hp), mm = mdot(hm, hm);
  const double rho = (mp > mm ? mp : mm) / sh;
  o.v[4] = rho > 0.0 ? rho : 0.0;
  bp /= 2.0 * sum;
  bm /= 2.0 * sum;
  o.v[5] = bp + bm;
  o.v[6] = bp > bm ? bp : bm;
  // Durham, E-scheme
  if (np >= 3) {
    const double inv_s = 1.0 / sh;
    double UX[M], UY[M], UZ[M];
#pragma unroll
    for (int a = 0; a < M; ++a) {
      UX[a] = UY[a] = UZ[a] = 0.0;
      if (a < np) {
        const double l = len3(X[a], Y[a], Z[a]);
        UX[a] = X[a] / l;
        UY[a] = Y[a] / l;
        UZ[a] = Z[a] / l;
      }
    }
    uint32_t alive = (1u << np) - 1u;
    for (int m = np; m > 2; --m) {
      double ymin = 0.0;
      int ia = -1, ib = -1;
#pragma unroll 1
      for (int a = 0; a + 1 < np; ++a) {
        if (!(alive >> a & 1u)) continue;
        double ea = 0.0, uxa = 0.0, uya = 0.0, uza = 0.0;
#pragma unroll
        for (int q = 0; q < M; ++q)
          if (q == a) { ea = E[q]; uxa = UX[q]; uya = UY[q]; uza = UZ[q]; }
#pragma unroll
        for (int b = 1; b < M; ++b) {
          if (b >= wmax) break;
          if (b > a && (alive >> b & 1u)) {
            const double dx = uxa - UX[b], dy = uya - UY[b], dz = uza - UZ[b];
            const double d2 = (dx * dx + dy * dy) + dz * dz;
            const double em = ea < E[b] ? ea : E[b];
            const double y = em * em * d2 * inv_s;
            if (ia < 0 || y < ymin) {
              ymin = y;
              ia = a;
              ib = b;
            }
          }
        }
      }
      if (m == 4) o.v[1] = ymin;
      if (m == 3) o.v[0] = ymin;
      if (m == 3) break;
      double eb = 0.0, xb = 0.0, yb = 0.0, zb = 0.0;
#pragma unroll
      for (int b = 0; b < M; ++b)
        if (b == ib) { eb = E[b]; xb = X[b]; yb = Y[b]; zb = Z[b]; }
#pragma unroll
      for (int a = 0; a < M; ++a) {
        if (a == ia) {
          E[a] += eb;
          X[a] += xb;
          Y[a] += yb;
          Z[a] += zb;
          const double l = len3(X[a], Y[a], Z[a]);
          UX[a] = X[a] / l;
          UY[a] = Y[a] / l;
          UZ[a] = Z[a] / l;
        }
      }
      alive &= ~(1u << ib);
    }
  }
  return o;
}

__device__ __forceinline__ double hist_lo(int h) {
  return h < 2 ? -4.3 : (h == 7 ? -1.0 : 0.0);
}
__device__ __forceinline__ double hist_hi(int h) {
  return h < 2 ? -0.3 : (h == 3 ? 1.0 : (h == 6 ? 0.35 : (h == 7 ? 1.0 : 0.5)));
}

// Scales of the fixed-point histogram: a weight w is held as the integer
// nearest to w 2^fw, w^2 as the one nearest to w^2 2^fw2, with 2^e above
// the launch's largest |w| and L = ceil(log2 n), so that no sum over the
// launch's n events leaves [-2^62, 2^62].
struct FixScale {
  int fw, fw2;
};

__device__ __forceinline__ FixScale fix_scale(const Scratch& sc) {
  const double m = __longlong_as_double((long long)*sc.wmax);
  int e = 0;
  (void)frexp(m, &e);  // m < 2^e (e = 0 for m = 0)
  return FixScale{62 - (int)sc.lbits - e, 62 - (int)sc.lbits - 2 * e};
}

// Fill one event into a histogram set [kNObs][kNHCol][3], in LDS or a
// global copy: FP64 sums, or (fx non-null) the fixed-point sums of
// fix_scale in the same words.
__device__ __forceinline__ void hist_fill(double* lh, const ObsOut& o, double w, double cos_theta,
                                              const FixScale* fx = nullptr) {
  double vals[kNObs];
  vals[0] = o.v[0] > 0.0 ? log10(o.v[0]) : -INFINITY;
  vals[1] = o.v[1] > 0.0 ? log10(o.v[1]) : -INFINITY;
  for (int h = 2; h < 7; ++h) vals[h] = o.v[h];
  vals[7] = cos_theta;
  unsigned long long qw = 0, qw2 = 0;
  if (fx) {
    qw = (unsigned long long)llrint(ldexp(w, fx->fw));
    qw2 = (unsigned long long)llrint(ldexp(w * w, fx->fw2));
  }
#pragma unroll
  for (int h = 0; h < kNObs; ++h) {
    const int b = bin_of(vals[h], hist_lo(h), hist_hi(h));
    double* cell = &lh[3 * (kNHCol * h + b)];
    if (fx) {
      unsigned long long* ic = reinterpret_cast<unsigned long long*>(cell);
      atomicAdd(&ic[0], qw);
      atomicAdd(&ic[1], qw2);
      atomicAdd(&ic[2], 1ull);
    } else {
      atomicAdd(&cell[0], w);
      atomicAdd(&cell[1], w * w);
      atomicAdd(&cell[2], 1.0);
    }
  }
}

// One LDS histogram set into this block's copy of the global one (block b:
// copy b mod kHistCopies): FP64 atomics, or integer atomics into the
// fixed-point cells.
__device__ __forceinline__ void hist_flush(const double* lh, const Scratch& sc, bool fixed, uint32_t t0,
                                           uint32_t step) {
  const unsigned long long* lq = reinterpret_cast<const unsigned long long*>(lh);
  const uint32_t c0 = (blockIdx.x % kHistCopies) * (uint32_t)kHistDoubles;
  for (uint32_t a = t0; a < (uint32_t)kHistDoubles; a += step) {
    if (fixed) {
      const unsigned long long q = lq[a];  // integer words: never read as doubles
      if (q) atomicAdd(&sc.ihist[c0 + a], q);
    } else {
      const double v = lh[a];
      if (v != 0.0) unsafeAtomicAdd(&sc.hcopy[c0 + a], v);
    }
  }
}

}  // namespace vsh
