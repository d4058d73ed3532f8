// pp_update.h -- per-particle update after the field sum (shared by the
// combine kernel and the fused small-bunch kernel): field output, the
// acceleration a = (q/m) E of Eqs. (D)/(F), the kick of Eq. (H) and the next
// step's drift of Eq. (G) with the source pack.  All FP64; the arithmetic of
// Eqs. (G)/(H) keeps its printed evaluation order (no contraction).
#pragma once

#include "pp_internal.h"

namespace ppk {

__device__ __forceinline__ double drift1(double r, double v, double acc, double dt) {
#pragma clang fp contract(off)
  return r + v * dt + acc * dt * dt / 2.0;
}

__device__ __forceinline__ double kick1(double v, double a0, double a1, double dt) {
#pragma clang fp contract(off)
  return v + (a0 + a1) * dt / 2.0;
}

// mirror of one particle: u = (r - origin) * scale, hi = fl32(u), lo = fl32(u - hi)
__device__ __forceinline__ void mirror1(double ox, double oy, double oz, double scale, int64_t i, double x, double y,
                                        double z, float* xh, float* yh, float* zh, float* xl, float* yl, float* zl) {
  const double ux = (x - ox) * scale;
  const double uy = (y - oy) * scale;
  const double uz = (z - oz) * scale;
  const float hx = (float)ux, hy = (float)uy, hz = (float)uz;
  xh[i] = hx; yh[i] = hy; zh[i] = hz;
  xl[i] = (float)(ux - (double)hx);
  yl[i] = (float)(uy - (double)hy);
  zl[i] = (float)(uz - (double)hz);
}

// The update of particle i of bunch B from its summed field S (ex, ey, ez,
// in the bunch's units: E = kE S) and potential sum ph.  FIN_KICK_DRIFT also
// writes the next positions' source copy: the mixed mirror (xh..zl) and, where
// given, the FP64 source copy (sx, sy, sz).
template <bool MIXED, int MODE>
__device__ __forceinline__ void update_particle(const FinalArgs& a, const BunchDev& B, int64_t i, double ex,
                                                double ey, double ez, double ph, bool want_phi) {
  // Everything the update reads, loaded before its first store: read after
  // them, the loads of x would wait for the stores of v and the bunch
  // constants for the stores of x (the compiler cannot rule out aliasing),
  // each a further round trip to memory.
  const double dt = B.dt, kE = B.kE;
  double ox = 0.0, oy = 0.0, oz = 0.0, scale = 0.0;
  double qi = 0.0, mi = 1.0, v0x = 0.0, v0y = 0.0, v0z = 0.0, a0x = 0.0, a0y = 0.0, a0z = 0.0;
  double rx = 0.0, ry = 0.0, rz = 0.0;
  if (MODE != FIN_FIELD) { qi = a.q[i]; mi = a.m[i]; }
  if (MODE == FIN_KICK || MODE == FIN_KICK_DRIFT) {
    v0x = a.vx[i]; v0y = a.vy[i]; v0z = a.vz[i];
    a0x = a.ax[i]; a0y = a.ay[i]; a0z = a.az[i];
  }
  if (MODE == FIN_KICK_DRIFT) {
    rx = a.x[i]; ry = a.y[i]; rz = a.z[i];
    if (MIXED) { ox = B.origin[0]; oy = B.origin[1]; oz = B.origin[2]; scale = B.scale; }
  }
  ex *= kE; ey *= kE; ez *= kE;
  if (MODE == FIN_FIELD) {
    if (a.ex) { a.ex[i] = ex; a.ey[i] = ey; a.ez[i] = ez; }
    if (want_phi) a.phi[i] = ph * B.kPhi;
    return;
  }
  const double qm = qi / mi;
  const double nax = ex * qm, nay = ey * qm, naz = ez * qm;
  if (MODE == FIN_KICK || MODE == FIN_KICK_DRIFT) {
    const double vx = kick1(v0x, a0x, nax, dt);
    const double vy = kick1(v0y, a0y, nay, dt);
    const double vz = kick1(v0z, a0z, naz, dt);
    a.vx[i] = vx; a.vy[i] = vy; a.vz[i] = vz;
    if (MODE == FIN_KICK_DRIFT) {
      // the next step's drift (Eq. (G)) with the velocity and acceleration just stored
      const double x = drift1(rx, vx, nax, dt);
      const double y = drift1(ry, vy, nay, dt);
      const double z = drift1(rz, vz, naz, dt);
      a.x[i] = x; a.y[i] = y; a.z[i] = z;
      if (MIXED) mirror1(ox, oy, oz, scale, i, x, y, z, a.xh, a.yh, a.zh, a.xl, a.yl, a.zl);
      else if (a.sx) { a.sx[i] = x; a.sy[i] = y; a.sz[i] = z; }
    }
  }
  a.ax[i] = nax; a.ay[i] = nay; a.az[i] = naz;
}

}  // namespace ppk
