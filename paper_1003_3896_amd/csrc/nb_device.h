// Device helpers for the gfx950 kernels of libnbody.
#pragma once
#include "nb_internal.h"

namespace nb {

// Fixed-order reduction of V doubles per thread over the block (a shuffle tree inside each wave,
// then the waves in order); result valid in thread 0.  sh needs [V][kBlock / 64].
template <int V>
__device__ __forceinline__ void block_reduce(double (&val)[V], double (*sh)[kBlock]) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1)
#pragma unroll
    for (int q = 0; q < V; ++q) val[q] += __shfl_down(val[q], m);
  __syncthreads();  // sh is free (a previous reduction has been read)
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < V; ++q) sh[q][wave] = val[q];
  __syncthreads();
  if (t == 0)
#pragma unroll
    for (int q = 0; q < V; ++q) {
      double s = sh[q][0];
      for (int w = 1; w < kBlock / 64; ++w) s += sh[q][w];
      val[q] = s;
    }
}

// Minima and maxima of V values per thread over the block; result valid in thread 0.
template <int V>
__device__ __forceinline__ void block_minmax(double (&mn)[V], double (&mx)[V], double (*sh)[kBlock]) {
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1)
#pragma unroll
    for (int q = 0; q < V; ++q) {
      mn[q] = fmin(mn[q], __shfl_down(mn[q], m));
      mx[q] = fmax(mx[q], __shfl_down(mx[q], m));
    }
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < V; ++q) {
      sh[q][wave] = mn[q];
      sh[V + q][wave] = mx[q];
    }
  __syncthreads();
  if (t == 0)
#pragma unroll
    for (int q = 0; q < V; ++q)
      for (int w = 1; w < kBlock / 64; ++w) {
        mn[q] = fmin(mn[q], sh[q][w]);
        mx[q] = fmax(mx[q], sh[V + q][w]);
      }
}

// External galaxy field at (X,Y,Z) in FP64 (the F_ext term of Eq. 3), acceleration = -grad Phi:
// model 0, Hernquist bulge + Miyamoto-Nagai disk + logarithmic halo; model 1, the Allen & Santillan
// (1991) Galaxy (a spherical bulge Phi = -G Mb / sqrt(r^2 + ab^2), the same disk, and a spherical
// halo of mass M(r) = Mh (r/ah)^2.02 / (1 + (r/ah)^1.02) inside r, constant beyond rcut); both with
// an optional softened point mass at the centre (the black hole of Sect. 6.2).  ALL_MODELS = false
// compiles model 0 only: the pair kernel never finishes a particle in model 1's field (those
// clusters are finished by the combine pass), and model 1's transcendental functions would take
// registers there.

// Model 1's halo: the mass inside min(r, rcut).
__device__ __forceinline__ double as91_halo_mass(const Galaxy& g, double r) {
  const double s = fmin(r, g.rcut) / g.ah;
  const double q = pow(s, 1.02);
  return g.Mh * s * q / (1.0 + q);
}

template <bool ALL_MODELS>
__device__ __forceinline__ void galaxy_accel(const Galaxy& g, double G, double X, double Y, double Z, double& ax,
                                             double& ay, double& az) {
  const double R2 = X * X + Y * Y;
  const double r2 = R2 + Z * Z;
  const double r = sqrt(r2);
  double fb, fh;  // |grad Phi_b| / r and |grad Phi_h| / r
  if (ALL_MODELS && g.model == kGalaxyAllenSantillan) {
    const double q = r2 + g.ab * g.ab;
    fb = G * g.Mb / (q * sqrt(q));
    fh = r > 0.0 ? G * as91_halo_mass(g, r) / (r2 * r) : 0.0;  // the field of the mass inside r
  } else {
    const double rb = r + g.ab;
    fb = r > 0.0 ? G * g.Mb / (r * rb * rb) : 0.0;
    fh = g.vh * g.vh / (r2 + g.dh * g.dh);
  }
  const double zs = sqrt(Z * Z + g.bd * g.bd);
  const double as = g.ad + zs;
  const double D2 = R2 + as * as;
  const double fd = G * g.Md / (D2 * sqrt(D2));                // (1/R) dPhi_d/dR
  const double fz = fd * as / zs;                               // (1/z) dPhi_d/dz
  const double q2 = r2 + g.ebh * g.ebh;
  const double fbh = g.Mbh > 0.0 ? G * g.Mbh / (q2 * sqrt(q2)) : 0.0;  // (1/r) dPhi_bh/dr
  const double fxy = fb + fd + fh + fbh;
  ax = -fxy * X;
  ay = -fxy * Y;
  az = -(fb + fz + fh + fbh) * Z;
}

// Model 1's halo potential: -G M(r)/r minus the work against the field of the mass inside from r out
// to rcut, G Mh / (1.02 ah) [H(rcut) - H(r)] with H(s) = ln(1 + (s/ah)^1.02) - 1.02 / (1 + (s/ah)^1.02),
// the closed form of that integral; beyond rcut the point-mass potential of M(rcut).
__device__ __forceinline__ double as91_halo_potential(const Galaxy& g, double G, double r) {
  if (r >= g.rcut) return -G * as91_halo_mass(g, g.rcut) / r;
  const double qc = pow(g.rcut / g.ah, 1.02), q = pow(r / g.ah, 1.02);
  const double Hc = log(1.0 + qc) - 1.02 / (1.0 + qc), H = log(1.0 + q) - 1.02 / (1.0 + q);
  const double inner = r > 0.0 ? -G * as91_halo_mass(g, r) / r : 0.0;  // M(r) ~ r^2.02 at the centre
  return inner - G * g.Mh / (1.02 * g.ah) * (Hc - H);
}

__device__ __forceinline__ double galaxy_potential(const Galaxy& g, double G, double X, double Y, double Z) {
  const double R2 = X * X + Y * Y;
  const double r2 = R2 + Z * Z;
  const double r = sqrt(r2);
  const double zs = sqrt(Z * Z + g.bd * g.bd);
  const double as = g.ad + zs;
  const double pbh = g.Mbh > 0.0 ? -G * g.Mbh / sqrt(r2 + g.ebh * g.ebh) : 0.0;
  const double pd = -G * g.Md / sqrt(R2 + as * as);
  if (g.model == kGalaxyAllenSantillan)
    return -G * g.Mb / sqrt(r2 + g.ab * g.ab) + pd + as91_halo_potential(g, G, r) + pbh;
  return -G * g.Mb / (r + g.ab) + pd + 0.5 * g.vh * g.vh * log(r2 + g.dh * g.dh) + pbh;
}

// 1/sqrt(x) in FP64: the hardware estimate (relative error ~2^-24) refined by one
// third-order Newton step y' = y + y e (1/2 + 3/8 e), e = 1 - x y^2 (error O(e^3)).
__device__ __forceinline__ double rsqrt_f64(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  const double h = x * y;
  const double e = fma(-h, y, 1.0);
  const double t = fma(0.375, e, 0.5);
  return fma(y * e, t, y);
}

// j-record of particle gi as the pair kernels consume it:
//   NB_FP32   (x, y, z, m) rounded to FP32 (absolute coordinates)
//   NB_FP32C  (x - ref, m) rounded to FP32, ref = the cluster's FP64 centre of mass
//   NB_FP32DS hi = fl32(x - ref), lo = fl32((x - ref) - hi)   (double-single coordinates)
//   NB_FP64   (x, y, z, m) in FP64 (absolute)
__device__ __forceinline__ void record32(const Args& a, long long gi, const double4& ref, float4& hi, float4& lo) {
  const double x = a.pos[3 * gi], y = a.pos[3 * gi + 1], z = a.pos[3 * gi + 2];
  const float m = (float)a.mass[gi];
  if (a.prec == 0) {
    hi = make_float4((float)x, (float)y, (float)z, m);
    lo = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    return;
  }
  const double dx = x - ref.x, dy = y - ref.y, dz = z - ref.z;
  const float hx = (float)dx, hy = (float)dy, hz = (float)dz;
  hi = make_float4(hx, hy, hz, m);
  lo = make_float4((float)(dx - (double)hx), (float)(dy - (double)hy), (float)(dz - (double)hz), 0.0f);
}

__device__ __forceinline__ double4 record64(const Args& a, long long gi) {
  return make_double4(a.pos[3 * gi], a.pos[3 * gi + 1], a.pos[3 * gi + 2], a.mass[gi]);
}

// Epilogue of one particle: scale by G, add the galaxy field (unless the pass wants the internal
// acceleration alone), store, optional kick.  ALL_MODELS: as in galaxy_accel.
template <bool ALL_MODELS>
__device__ __forceinline__ void finish_particle(const Args& a, const DevCluster& c, int cluster, long long gi,
                                                double ax, double ay, double az, bool round32, int kick) {
  ax *= a.G;
  ay *= a.G;
  az *= a.G;
  if (round32) {
    ax = (float)ax;
    ay = (float)ay;
    az = (float)az;
  }
  if ((c.flags & kFlagField) && !a.internal_only) {
    double ex, ey, ez;
    galaxy_accel<ALL_MODELS>(a.gal, a.G, a.pos[3 * gi], a.pos[3 * gi + 1], a.pos[3 * gi + 2], ex, ey, ez);
    ax += ex;
    ay += ey;
    az += ez;
    if (round32) {
      ax = (float)ax;
      ay = (float)ay;
      az = (float)az;
    }
  }
  if (a.acc) {
    a.acc[3 * gi] = ax;
    a.acc[3 * gi + 1] = ay;
    a.acc[3 * gi + 2] = az;
  }
  if (kick) {
    const double kp = a.coef ? a.coef[3 * cluster + 2] : a.kick_post;
    double* v = a.vel + 3 * gi;
    if (round32) {
      v[0] = fmaf((float)kp, (float)ax, (float)v[0]);
      v[1] = fmaf((float)kp, (float)ay, (float)v[1]);
      v[2] = fmaf((float)kp, (float)az, (float)v[2]);
    } else {
      v[0] = fma(kp, ax, v[0]);
      v[1] = fma(kp, ay, v[1]);
      v[2] = fma(kp, az, v[2]);
    }
  }
}

}  // namespace nb
