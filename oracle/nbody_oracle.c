/*
 * nbody_oracle.c -- plain, slow, FP64 CPU oracle for the direct-summation N-body hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or helper with the HIP path
 * and must never be called from it.
 *
 * What it computes (NBSymple, Capuzzo-Dolcetta, Mastrobuono-Battisti & Maschietti, New Astronomy):
 *   - softened pairwise gravitational acceleration, Sect. 2 Eq. 5 (with the j = i term left out,
 *     which Eq. 2 requires and which also makes eps = 0 well defined), and the softened potential
 *     of Eq. 4 summed over j != i;
 *   - an analytic external field (Sect. 3, Eq. 3 term F_ext): Hernquist bulge + Miyamoto-Nagai
 *     disk + logarithmic halo, closed forms from Binney & Tremaine (the paper names the Allen &
 *     Santillan bulge/disk/halo model without printing it);
 *   - energy, linear and angular momentum and external torque (Sect. 5.1, Eqs. 8-10), and the
 *     mass-weighted sum of the internal accelerations (zero by the antisymmetry of Eq. 2);
 *   - the 2nd-order leapfrog (Sect. 3.1) in kick-drift-kick form and the 6th-order symplectic
 *     integrator of Sect. 3.1 as a 7-stage symmetric composition of leapfrogs (Yoshida 1990,
 *     solution A), with adjacent half-kicks inside one step merged.
 *
 * Conventions: G, eps and the galaxy parameters are arguments; positions/velocities/accelerations
 * are row-major (n,3) doubles; potentials are negative for bound systems (Phi = -U of Eq. 4);
 * acceleration = -grad Phi.
 *
 * Every sum runs over j in ascending order with Neumaier compensation, so the oracle's own
 * rounding error (~1e-16 relative to the sum of absolute values) is far below any tolerance that
 * is checked against it.  Build with -O2 -ffp-contract=off so that no FMA contraction changes the
 * arithmetic from what is written here.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Neumaier (improved Kahan-Babuska) running sum: s + c is the compensated total. */
typedef struct { double s, c; } nsum;

static inline void nsum_add(nsum* a, double x) {
  double t = a->s + x;
  if (fabs(a->s) >= fabs(x))
    a->c += (a->s - t) + x;
  else
    a->c += (x - t) + a->s;
  a->s = t;
}
static inline double nsum_get(const nsum* a) { return a->s + a->c; }

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void oracle_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

/*
 * Softened internal acceleration and potential (Sect. 2, Eqs. 4-5):
 *   a_i   =  G sum_{j != i} m_j d_ij / (|d_ij|^2 + eps^2)^{3/2},   d_ij = x_j - x_i
 *   phi_i = -G sum_{j != i} m_j / sqrt(|d_ij|^2 + eps^2)
 *   absa_i=  G sum_{j != i} m_j |d_ij| / (|d_ij|^2 + eps^2)^{3/2}   (sum of pair magnitudes; the
 *            natural scale for the rounding error of any evaluation of the sum)
 * Any of acc/pot/absa may be NULL.  Rows [i0, i1) are evaluated against all n sources.
 */
void oracle_accel_range(int64_t n, int64_t i0, int64_t i1, const double* pos, const double* mass,
                        double G, double eps, double* acc, double* pot, double* absa) {
  const double e2 = eps * eps;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = i0; i < i1; ++i) {
    const double xi = pos[3 * i], yi = pos[3 * i + 1], zi = pos[3 * i + 2];
    nsum ax = {0, 0}, ay = {0, 0}, az = {0, 0}, ph = {0, 0}, ab = {0, 0};
    for (int64_t j = 0; j < n; ++j) {
      if (j == i) continue;
      const double dx = pos[3 * j] - xi;
      const double dy = pos[3 * j + 1] - yi;
      const double dz = pos[3 * j + 2] - zi;
      const double r2 = dx * dx + dy * dy + dz * dz + e2;
      const double inv = 1.0 / sqrt(r2);
      const double inv3 = inv * inv * inv;
      const double s = mass[j] * inv3;
      nsum_add(&ax, s * dx);
      nsum_add(&ay, s * dy);
      nsum_add(&az, s * dz);
      nsum_add(&ph, mass[j] * inv);
      nsum_add(&ab, s * sqrt(dx * dx + dy * dy + dz * dz));
    }
    if (acc) {
      acc[3 * (i - i0)] = G * nsum_get(&ax);
      acc[3 * (i - i0) + 1] = G * nsum_get(&ay);
      acc[3 * (i - i0) + 2] = G * nsum_get(&az);
    }
    if (pot) pot[i - i0] = -G * nsum_get(&ph);
    if (absa) absa[i - i0] = G * nsum_get(&ab);
  }
}

void oracle_accel(int64_t n, const double* pos, const double* mass, double G, double eps, double* acc,
                  double* pot, double* absa) {
  oracle_accel_range(n, 0, n, pos, mass, G, eps, acc, pot, absa);
}

/*
 * External galactic field.  gal = {Mb, ab, Md, ad, bd, vh, dh, Mbh, ebh, model, Mh, ah, rcut}.
 * model 0:
 *   Hernquist bulge:      Phi_b = -G Mb / (r + ab)
 *   Miyamoto-Nagai disk:  Phi_d = -G Md / sqrt(R^2 + (ad + sqrt(z^2 + bd^2))^2)
 *   logarithmic halo:     Phi_h =  vh^2 / 2 * ln(r^2 + dh^2)
 * model 1, the Galaxy of Allen & Santillan (1991) that Sect. 3 names (spherical bulge and halo,
 * axisymmetric disk):
 *   bulge:                Phi_b = -G Mb / sqrt(r^2 + ab^2)
 *   Miyamoto-Nagai disk:  as in model 0
 *   halo:                 mass inside r, M(r) = Mh (r/ah)^2.02 / (1 + (r/ah)^1.02), for r < rcut and
 *                         M(rcut) beyond; the potential is -G M(r)/r plus the integral of G M(s)/s^2
 *                         from r to rcut, which is -G Mh / (1.02 ah) [H(rcut) - H(r)] with
 *                         H(s) = ln(1 + (s/ah)^1.02) - 1.02 / (1 + (s/ah)^1.02); beyond rcut
 *                         -G M(rcut) / r
 * both models:
 *   central black hole:   Phi_bh = -G Mbh / sqrt(r^2 + ebh^2)  (a fixed point mass at the galaxy
 *                         centre, softened like a star; the massive point of Sect. 6.2)
 * with R^2 = x^2 + y^2, r^2 = R^2 + z^2.  Acceleration is -grad Phi, written out per component.
 * acc/phi may be NULL.
 */
static double as91_halo_mass(double r, double Mh, double ah, double rcut) {
  const double s = r < rcut ? r : rcut;
  const double q = pow(s / ah, 1.02);
  return Mh * (s / ah) * q / (1.0 + q);
}

static double as91_H(double s, double ah) {
  const double q = pow(s / ah, 1.02);
  return log(1.0 + q) - 1.02 / (1.0 + q);
}
static void ext_one(const double* x, double G, const double* gal, double* a, double* phi) {
  const double Mb = gal[0], ab = gal[1], Md = gal[2], ad = gal[3], bd = gal[4], vh = gal[5], dh = gal[6];
  const double Mbh = gal[7], ebh = gal[8];
  const int as91 = gal[9] == 1.0;
  const double Mh = gal[10], ah = gal[11], rcut = gal[12];
  const double X = x[0], Y = x[1], Z = x[2];
  const double R2 = X * X + Y * Y;
  const double r2 = R2 + Z * Z;
  const double r = sqrt(r2);
  /* bulge: grad Phi_b = G Mb / (r + ab)^2 * xhat (model 0), G Mb r / (r^2 + ab^2)^(3/2) * xhat (model 1) */
  double gb = 0.0; /* grad magnitude over r */
  if (as91)
    gb = G * Mb / pow(r2 + ab * ab, 1.5);
  else if (r > 0.0)
    gb = G * Mb / (r * (r + ab) * (r + ab));
  /* disk */
  const double s = sqrt(Z * Z + bd * bd);
  const double As = ad + s;
  const double D2 = R2 + As * As;
  const double D = sqrt(D2);
  const double D3 = D2 * D;
  const double gdR = G * Md / D3;             /* d Phi_d / dx = gdR * x */
  const double gdz = G * Md * As / (D3 * s);  /* d Phi_d / dz = gdz * z */
  /* halo: d Phi_h / dx = gh * x; in model 1 gh = G M(r) / r^3 (the field of the mass inside r) */
  double gh;
  if (as91)
    gh = r > 0.0 ? G * as91_halo_mass(r, Mh, ah, rcut) / (r2 * r) : 0.0;
  else
    gh = vh * vh / (r2 + dh * dh);
  /* black hole: d Phi_bh / dx = G Mbh x / (r^2 + ebh^2)^(3/2) */
  const double q2 = r2 + ebh * ebh;
  const double gbh = Mbh > 0.0 ? G * Mbh / (q2 * sqrt(q2)) : 0.0;
  if (a) {
    a[0] = -(gb * X + gdR * X + gh * X + gbh * X);
    a[1] = -(gb * Y + gdR * Y + gh * Y + gbh * Y);
    a[2] = -(gb * Z + gdz * Z + gh * Z + gbh * Z);
  }
  if (phi) {
    const double pb = as91 ? -G * Mb / sqrt(r2 + ab * ab) : -G * Mb / (r + ab);
    const double pd = -G * Md / D;
    double ph;
    if (!as91)
      ph = 0.5 * vh * vh * log(r2 + dh * dh);
    else if (r >= rcut)
      ph = -G * as91_halo_mass(rcut, Mh, ah, rcut) / r;
    else /* M(r)/r -> 0 at the centre, since M(r) ~ r^2.02 */
      ph = (r > 0.0 ? -G * as91_halo_mass(r, Mh, ah, rcut) / r : 0.0) -
           G * Mh / (1.02 * ah) * (as91_H(rcut, ah) - as91_H(r, ah));
    const double pbh = Mbh > 0.0 ? -G * Mbh / sqrt(q2) : 0.0;
    *phi = pb + pd + ph + pbh;
  }
}

void oracle_ext_field(int64_t n, const double* pos, double G, const double* gal, double* acc, double* phi) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) ext_one(pos + 3 * i, G, gal, acc ? acc + 3 * i : 0, phi ? phi + i : 0);
}

/* total acceleration (internal + optional external), as used by the integrators (Eq. 3) */
static void total_accel(int64_t n, const double* pos, const double* mass, double G, double eps, int field,
                        const double* gal, double* acc) {
  oracle_accel(n, pos, mass, G, eps, acc, 0, 0);
  if (field) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      double ae[3];
      ext_one(pos + 3 * i, G, gal, ae, 0);
      acc[3 * i] += ae[0];
      acc[3 * i + 1] += ae[1];
      acc[3 * i + 2] += ae[2];
    }
  }
}

/*
 * Diagnostics of Sect. 5.1 (Eqs. 8-10), plus the internal force sum of Sect. 2.  out[20]:
 *   0 K = 1/2 sum m v^2        1 W = 1/2 sum m_i phi_i (pairs j != i, softened)
 *   2 Uext = sum m Phi_ext     3 E = K + W + Uext
 *   4..6 P = sum m v           7..9 L = sum m x cross v
 *   10..12 torque = sum m x cross a_ext(x)  (Eq. 8, with F_ext an acceleration as in Eq. 3)
 *   13 M = sum m
 *   14..16 F = sum m a_int     (the pair forces of Eq. 2 are antisymmetric, so F = 0 exactly and
 *                              only rounding remains)
 *   17 |F|                     18 sum m |a_int|  (the scale |F| is to be compared with)
 *   19 zero
 * scratch: 4 n doubles (internal accelerations, then pair potentials).
 */
void oracle_energy(int64_t n, const double* pos, const double* vel, const double* mass, double G, double eps,
                   int field, const double* gal, double* out, double* scratch) {
  double* acc = scratch;
  double* pot = scratch + 3 * n;
  oracle_accel(n, pos, mass, G, eps, acc, pot, 0);
  nsum K = {0, 0}, W = {0, 0}, U = {0, 0}, P[3] = {{0, 0}, {0, 0}, {0, 0}}, L[3] = {{0, 0}, {0, 0}, {0, 0}},
       T[3] = {{0, 0}, {0, 0}, {0, 0}}, M = {0, 0}, F[3] = {{0, 0}, {0, 0}, {0, 0}}, A = {0, 0};
  for (int64_t i = 0; i < n; ++i) {
    const double m = mass[i];
    const double* x = pos + 3 * i;
    const double* v = vel + 3 * i;
    const double* a = acc + 3 * i;
    nsum_add(&K, 0.5 * m * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
    nsum_add(&W, 0.5 * m * pot[i]);
    for (int c = 0; c < 3; ++c) nsum_add(&P[c], m * v[c]);
    for (int c = 0; c < 3; ++c) nsum_add(&F[c], m * a[c]);
    nsum_add(&A, m * sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]));
    nsum_add(&L[0], m * (x[1] * v[2] - x[2] * v[1]));
    nsum_add(&L[1], m * (x[2] * v[0] - x[0] * v[2]));
    nsum_add(&L[2], m * (x[0] * v[1] - x[1] * v[0]));
    nsum_add(&M, m);
    if (field) {
      double ae[3], ph;
      ext_one(x, G, gal, ae, &ph);
      nsum_add(&U, m * ph);
      nsum_add(&T[0], m * (x[1] * ae[2] - x[2] * ae[1]));
      nsum_add(&T[1], m * (x[2] * ae[0] - x[0] * ae[2]));
      nsum_add(&T[2], m * (x[0] * ae[1] - x[1] * ae[0]));
    }
  }
  memset(out, 0, 20 * sizeof(double));
  out[0] = nsum_get(&K);
  out[1] = nsum_get(&W);
  out[2] = nsum_get(&U);
  out[3] = out[0] + out[1] + out[2];
  for (int c = 0; c < 3; ++c) {
    out[4 + c] = nsum_get(&P[c]);
    out[7 + c] = nsum_get(&L[c]);
    out[10 + c] = nsum_get(&T[c]);
    out[14 + c] = nsum_get(&F[c]);
  }
  out[13] = nsum_get(&M);
  out[17] = sqrt(out[14] * out[14] + out[15] * out[15] + out[16] * out[16]);
  out[18] = nsum_get(&A);
}

/*
 * 6th-order symmetric composition (Sect. 3.1; coefficients of Yoshida 1990, solution A):
 *   S6(h) = S2(w3 h) S2(w2 h) S2(w1 h) S2(w0 h) S2(w1 h) S2(w2 h) S2(w3 h),  w0 = 1 - 2(w1+w2+w3)
 * where S2 is the kick-drift-kick leapfrog.  Merging the touching half-kicks of consecutive S2
 * inside one step gives 7 drifts and 8 kicks; the first kick reuses the acceleration that the
 * previous step ended with, so each step costs 7 new force evaluations.
 */
static const double W1 = -1.17767998417887;
static const double W2 = 0.235573213359357;
static const double W3 = 0.784513610477560;

void oracle_sym6_coefficients(double* drift7, double* kick8) {
  const double W0 = 1.0 - 2.0 * (W1 + W2 + W3);
  const double w[7] = {W3, W2, W1, W0, W1, W2, W3};
  for (int k = 0; k < 7; ++k) drift7[k] = w[k];
  kick8[0] = 0.5 * w[0];
  for (int k = 1; k < 7; ++k) kick8[k] = 0.5 * (w[k - 1] + w[k]);
  kick8[7] = 0.5 * w[6];
}

static void kick(int64_t n, double* vel, const double* acc, double c) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < 3 * n; ++i) vel[i] = vel[i] + c * acc[i];
}
static void drift(int64_t n, double* pos, const double* vel, double c) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < 3 * n; ++i) pos[i] = pos[i] + c * vel[i];
}

/*
 * Advance one isolated cluster by nsteps steps of size dt.
 *   integrator 0: leapfrog KDK  v += dt/2 a;  x += dt v;  a = A(x);  v += dt/2 a
 *   integrator 1: 6th-order composition above
 * acc holds A(x) on entry (the caller evaluates it once) and A(x_final) on return.
 * A(x) = internal softened acceleration + external field when field != 0.
 */
void oracle_step(int64_t n, double* pos, double* vel, const double* mass, double* acc, double G, double eps,
                 int field, const double* gal, double dt, int64_t nsteps, int integrator) {
  double D[7], Kc[8];
  int stages;
  if (integrator == 0) {
    D[0] = 1.0;
    Kc[0] = 0.5;
    Kc[1] = 0.5;
    stages = 1;
  } else {
    oracle_sym6_coefficients(D, Kc);
    stages = 7;
  }
  for (int64_t s = 0; s < nsteps; ++s) {
    for (int k = 0; k < stages; ++k) {
      kick(n, vel, acc, Kc[k] * dt);
      drift(n, pos, vel, D[k] * dt);
      total_accel(n, pos, mass, G, eps, field, gal, acc);
    }
    kick(n, vel, acc, Kc[stages] * dt);
  }
}

/* acceleration used by the integrators (internal + optional field), for the caller's first eval */
void oracle_total_accel(int64_t n, const double* pos, const double* mass, double G, double eps, int field,
                        const double* gal, double* acc) {
  total_accel(n, pos, mass, G, eps, field, gal, acc);
}
