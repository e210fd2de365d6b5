/*
 * fdtd_oracle.c -- plain, slow FP64 CPU implementation of imaginary-time FDTD
 * relaxation (Strickland & Yager-Elorriaga, "A Parallel Algorithm for Solving
 * the 3d Schroedinger Equation", arXiv:0904.0939).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the oracle that the HIP path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no code, header, table or
 * constant with the GPU library: every formula below is written again from the
 * paper.  Everything is double precision, plain loops, no blocking or fusion.
 * The only parallelism is an OpenMP loop over x-planes inside the update and
 * upsample sweeps; the arithmetic of each site does not depend on the thread
 * count, and every reduction is a serial loop in lattice order.
 *
 * Lattice convention (the paper fixes L = N a and measures r from the centre
 * of the lattice, Sec. III and Sec. VII.C/D): sites i = 0..N-1 per axis sit at
 *     x_i = (2 i - (N - 1)) * (a / 2),   a = L / N,
 * i.e. cell centred; the mirror i <-> N-1-i negates x exactly.  Ghost sites
 * i = -1 and i = N hold psi = 0 (Dirichlet, Sec. III and Sec. V).  Storage is
 * psi[(ix * N + iy) * N + iz], z fastest.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_IDX(N, x, y, z) ((((int64_t)(x) * (N)) + (y)) * (N) + (z))

/* Potential kinds.  The numbering is a convention the tests share with the GPU
 * library's public header (checked by a test); the formulas are restated here. */
enum {
  ORC_POT_CONST = 0,   /* V = p0 */
  ORC_POT_HO = 1,      /* V = (wx^2 x^2 + wy^2 y^2 + wz^2 z^2) / 2, p = {wx, wy, wz} */
  ORC_POT_COULOMB = 2, /* V = -p0 / r */
  ORC_POT_COULOMB_REG = 3, /* Eq. (coulombpot): 0 for r < a, -p0/r + p0/a for r >= a */
  ORC_POT_CORNELL = 4, /* V = -p0 / r + p1 r + p2 z^2 */
  ORC_POT_WELLS = 5,   /* HO(p0..p2) - sum_k A_k exp(-|r - c_k|^2 / (2 s_k^2)),
                          then 5 values per well: A, cx, cy, cz, s */
  ORC_POT_DODECA = 6   /* Sec. VII.E: V = p0 inside a regular dodecahedron, 0
                          outside; see orc_dodeca_inside */
};

/* Regular dodecahedron of Sec. VII.E in lattice units u = x / ((N - 1) a / 2),
 * so u = -1 is the first site and u = 1 the last one on each axis.  Its 20
 * vertices are (+-1, +-1, +-1)/phi, (0, +-1/phi^2, +-1), (+-1/phi^2, +-1, 0)
 * and (+-1, 0, +-1/phi^2), phi the golden ratio: the circumsphere has radius
 * sqrt(3)/phi, as the paper states (its printed list repeats a vertex family
 * with two coordinates exchanged; this is the regular solid its text
 * describes).  The 12 faces are perpendicular to the directions (0, +-phi,
 * +-1), (+-1, 0, +-phi), (+-phi, +-1, 0) (an icosahedron); each face plane
 * is at the largest projection of the vertices on its unit normal, reached by
 * exactly the 5 vertices of that face.  A point is inside
 * when its projection on every normal is at most that distance. */
static int orc_dodeca_inside(double ux, double uy, double uz) {
  const double phi = 0.5 * (1.0 + sqrt(5.0));
  const double vtx[20][3] = {
      {1 / phi, 1 / phi, 1 / phi},   {1 / phi, 1 / phi, -1 / phi},
      {1 / phi, -1 / phi, 1 / phi},  {1 / phi, -1 / phi, -1 / phi},
      {-1 / phi, 1 / phi, 1 / phi},  {-1 / phi, 1 / phi, -1 / phi},
      {-1 / phi, -1 / phi, 1 / phi}, {-1 / phi, -1 / phi, -1 / phi},
      {0, 1 / (phi * phi), 1},       {0, 1 / (phi * phi), -1},
      {0, -1 / (phi * phi), 1},      {0, -1 / (phi * phi), -1},
      {1 / (phi * phi), 1, 0},       {1 / (phi * phi), -1, 0},
      {-1 / (phi * phi), 1, 0},      {-1 / (phi * phi), -1, 0},
      {1, 0, 1 / (phi * phi)},       {1, 0, -1 / (phi * phi)},
      {-1, 0, 1 / (phi * phi)},      {-1, 0, -1 / (phi * phi)}};
  const double nrm[6][3] = {{0, phi, 1}, {0, phi, -1}, {1, 0, phi},
                            {-1, 0, phi}, {phi, 1, 0}, {phi, -1, 0}};
  for (int f = 0; f < 6; ++f) {
    const double len = sqrt(nrm[f][0] * nrm[f][0] + nrm[f][1] * nrm[f][1] + nrm[f][2] * nrm[f][2]);
    double d = 0.0; /* face distance: the largest vertex projection */
    for (int v = 0; v < 20; ++v) {
      const double pr = (vtx[v][0] * nrm[f][0] + vtx[v][1] * nrm[f][1] + vtx[v][2] * nrm[f][2]) / len;
      if (pr > d) d = pr;
    }
    const double q = (ux * nrm[f][0] + uy * nrm[f][1] + uz * nrm[f][2]) / len;
    /* +n and -n faces at once; the solid is closed, with a relative slack of
     * 1e-12 so that sites exactly on a face (edge midpoints for odd N) are
     * inside whatever the last bit of the arithmetic */
    if (fabs(q) > d * (1.0 + 1e-12)) return 0;
  }
  return 1;
}

static double orc_coord(int i, int N, double a) {
  return (2.0 * (double)i - (double)(N - 1)) * (0.5 * a);
}

/* Evaluate an analytic potential at every site.  Returns 0, or -1 on bad input. */
int orc_potential(int kind, const double* p, int np, int N, double L, double* V) {
  const double a = L / (double)N;
  if (N < 1) return -1;
  if (kind == ORC_POT_WELLS && (np < 3 || (np - 3) % 5 != 0)) return -1;
  if ((kind == ORC_POT_HO) && np < 3) return -1;
  if ((kind == ORC_POT_COULOMB || kind == ORC_POT_COULOMB_REG || kind == ORC_POT_CONST) && np < 1)
    return -1;
  if (kind == ORC_POT_CORNELL && np < 3) return -1;
  if (kind == ORC_POT_DODECA && np < 1) return -1;
  const double half = 0.5 * (double)(N - 1) * a; /* u = x / half */
  for (int ix = 0; ix < N; ++ix) {
    const double x = orc_coord(ix, N, a);
    for (int iy = 0; iy < N; ++iy) {
      const double y = orc_coord(iy, N, a);
      for (int iz = 0; iz < N; ++iz) {
        const double z = orc_coord(iz, N, a);
        const double r = sqrt(x * x + y * y + z * z);
        double v = 0.0;
        switch (kind) {
          case ORC_POT_CONST: v = p[0]; break;
          case ORC_POT_HO:
            v = 0.5 * (p[0] * p[0] * x * x + p[1] * p[1] * y * y + p[2] * p[2] * z * z);
            break;
          case ORC_POT_COULOMB: v = -p[0] / r; break;
          case ORC_POT_COULOMB_REG: v = (r < a) ? 0.0 : (-p[0] / r + p[0] / a); break;
          case ORC_POT_CORNELL: v = -p[0] / r + p[1] * r + p[2] * z * z; break;
          case ORC_POT_WELLS: {
            v = 0.5 * (p[0] * p[0] * x * x + p[1] * p[1] * y * y + p[2] * p[2] * z * z);
            const int nw = (np - 3) / 5;
            for (int k = 0; k < nw; ++k) {
              const double* w = p + 3 + 5 * k;
              const double dx = x - w[1], dy = y - w[2], dz = z - w[3];
              const double d2 = dx * dx + dy * dy + dz * dz;
              v -= w[0] * exp(-d2 / (2.0 * w[4] * w[4]));
            }
            break;
          }
          case ORC_POT_DODECA:
            v = (N > 1 && orc_dodeca_inside(x / half, y / half, z / half)) ? p[0] : 0.0;
            break;
          default: return -1;
        }
        V[ORC_IDX(N, ix, iy, iz)] = v;
      }
    }
  }
  return 0;
}

/* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the n-th output (n >= 1) of
 * the generator seeded with s is mix(s + n * gamma).  Used counter-based: the
 * counter of a draw is (member << 36) + 2 * site + j, j in {0, 1}. */
static uint64_t orc_splitmix(uint64_t seed, uint64_t counter) {
  uint64_t z = seed + (counter + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

static double orc_unit(uint64_t r) { /* [0, 1) with 53 random bits */
  return (double)(r >> 11) * (1.0 / 9007199254740992.0);
}

int orc_reimpose(int N, uint32_t parity, double* psi);

/* Random initial condition (Sec. III: random numbers of amplitude one) followed
 * by the symmetry operators of Sec. IV.  kind 0: uniform in [-1, 1); kind 1:
 * unit Gaussian (Box-Muller).  parity holds 2 bits per axis (x: bits 0-1,
 * y: 2-3, z: 4-5): 0 free, 1 S (copy), 2 A (copy with sign flip).  The copy
 * goes from the lower half i < N/2 onto i' = N-1-i; for odd N the mid plane is
 * kept under S and zeroed under A.  Returns 0, or -1 on bad input. */
int orc_initial(uint64_t seed, uint32_t member, int kind, uint32_t parity, int N, double* psi) {
  if (N < 1 || (kind != 0 && kind != 1)) return -1;
  for (int ax = 0; ax < 3; ++ax)
    if (((parity >> (2 * ax)) & 3u) == 3u) return -1;
  const int64_t n3 = (int64_t)N * N * N;
  for (int64_t s = 0; s < n3; ++s) {
    const uint64_t base = ((uint64_t)member << 36) + 2u * (uint64_t)s;
    if (kind == 0) {
      psi[s] = 2.0 * orc_unit(orc_splitmix(seed, base)) - 1.0;
    } else {
      const double u1 = orc_unit(orc_splitmix(seed, base)) + 1.0 / 9007199254740992.0;
      const double u2 = orc_unit(orc_splitmix(seed, base + 1u));
      psi[s] = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
    }
  }
  return orc_reimpose(N, parity, psi);
}

/* The symmetry operators of Sec. IV applied to a state in place: for each
 * masked axis in turn (x, then y, then z), the lower half i < N/2 is copied
 * onto the mirror sites i' = N-1-i, with the sign flipped under A; for odd N
 * the mid plane is kept under S and zeroed under A.  The same operation makes
 * the symmetric initial state and, applied again during the relaxation,
 * reimposes the symmetry ("periodically", Sec. IV).  Returns 0, or -1 on a bad
 * parity word. */
int orc_reimpose(int N, uint32_t parity, double* psi) {
  if (N < 1 || (parity >> 6)) return -1;
  for (int ax = 0; ax < 3; ++ax)
    if (((parity >> (2 * ax)) & 3u) == 3u) return -1;
  /* one axis at a time, exactly as the copy is described */
  for (int ax = 0; ax < 3; ++ax) {
    const uint32_t m = (parity >> (2 * ax)) & 3u;
    if (m == 0) continue;
    const double sign = (m == 2u) ? -1.0 : 1.0;
    for (int ix = 0; ix < N; ++ix)
      for (int iy = 0; iy < N; ++iy)
        for (int iz = 0; iz < N; ++iz) {
          int c[3] = {ix, iy, iz};
          const int i = c[ax], mirror = N - 1 - i;
          if (i > mirror) { /* upper half: overwrite from the mirror site */
            c[ax] = mirror;
            psi[ORC_IDX(N, ix, iy, iz)] = sign * psi[ORC_IDX(N, c[0], c[1], c[2])];
          } else if (i == mirror && m == 2u) {
            psi[ORC_IDX(N, ix, iy, iz)] = 0.0;
          }
        }
  }
  return 0;
}

static double orc_at(const double* f, int N, int x, int y, int z) {
  if (x < 0 || y < 0 || z < 0 || x >= N || y >= N || z >= N) return 0.0; /* ghost */
  return f[ORC_IDX(N, x, y, z)];
}

/* a^2 * (sum over axes of D . Psi-hat), the 7-point Laplacian of Sec. III
 * without the 1/a^2.  Each axis term is (left + right) - 2 centre; the axes
 * are summed x, y, z. */
static double orc_lap_a2(const double* f, int N, int x, int y, int z) {
  const double c = f[ORC_IDX(N, x, y, z)];
  const double tx = (orc_at(f, N, x - 1, y, z) + orc_at(f, N, x + 1, y, z)) - 2.0 * c;
  const double ty = (orc_at(f, N, x, y - 1, z) + orc_at(f, N, x, y + 1, z)) - 2.0 * c;
  const double tz = (orc_at(f, N, x, y, z - 1) + orc_at(f, N, x, y, z + 1)) - 2.0 * c;
  return (tx + ty) + tz;
}

/* One imaginary-time step, Eq. (updateeq) with A and B as defined below it:
 *   psi'(r) = A psi(r) + (B dt / 2m) sum_i (D . Psi-hat)_i,
 *   A = (1 - dt V/2) / (1 + dt V/2),  B = 1 / (1 + dt V/2). */
void orc_step(int N, double L, double mass, double dt, const double* V, const double* in,
              double* out) {
  const double a = L / (double)N;
#pragma omp parallel for schedule(static)
  for (int ix = 0; ix < N; ++ix)
    for (int iy = 0; iy < N; ++iy)
      for (int iz = 0; iz < N; ++iz) {
        const int64_t s = ORC_IDX(N, ix, iy, iz);
        const double v = V[s];
        const double A = (1.0 - 0.5 * dt * v) / (1.0 + 0.5 * dt * v);
        const double B = 1.0 / (1.0 + 0.5 * dt * v);
        const double lap = orc_lap_a2(in, N, ix, iy, iz) / (a * a);
        out[s] = A * in[s] + (B * dt / (2.0 * mass)) * lap;
      }
}

/* H psi = -(1/2m) lap psi + V psi, the operator whose expectation value Eq.
 * (energy0) takes; used by the observables and the adjoint start. */
void orc_hpsi(int N, double L, double mass, const double* V, const double* psi, double* out) {
  const double a = L / (double)N;
  for (int ix = 0; ix < N; ++ix)
    for (int iy = 0; iy < N; ++iy)
      for (int iz = 0; iz < N; ++iz) {
        const int64_t s = ORC_IDX(N, ix, iy, iz);
        out[s] = -orc_lap_a2(psi, N, ix, iy, iz) / (2.0 * mass * a * a) + V[s] * psi[s];
      }
}

/* Observables of a state.  out = {norm2, E, kinetic, potential, r_rms, binding}
 *   norm2 = a^3 sum psi^2,
 *   E     = sum psi (H psi) / sum psi^2   (Eq. energysum; the sign there is
 *           printed reversed, the paper's own HO energy fixes it to <H>),
 *   kinetic, potential = the two parts of E,
 *   r_rms = sqrt(sum r^2 psi^2 / sum psi^2), r from the lattice centre,
 *   binding = E - v_inf (Eq. bindingenergy with constant V_inf). */
void orc_observables(int N, double L, double mass, const double* V, const double* psi,
                     double v_inf, double* out) {
  const double a = L / (double)N;
  double s0 = 0.0, kin = 0.0, pot = 0.0, r2 = 0.0;
  for (int ix = 0; ix < N; ++ix) {
    const double x = orc_coord(ix, N, a);
    for (int iy = 0; iy < N; ++iy) {
      const double y = orc_coord(iy, N, a);
      for (int iz = 0; iz < N; ++iz) {
        const double z = orc_coord(iz, N, a);
        const int64_t s = ORC_IDX(N, ix, iy, iz);
        const double p = psi[s];
        s0 += p * p;
        kin += p * (-orc_lap_a2(psi, N, ix, iy, iz) / (2.0 * mass * a * a));
        pot += p * V[s] * p;
        r2 += (x * x + y * y + z * z) * p * p;
      }
    }
  }
  out[0] = s0 * a * a * a;
  out[1] = (kin + pot) / s0;
  out[2] = kin / s0;
  out[3] = pot / s0;
  out[4] = sqrt(r2 / s0);
  out[5] = out[1] - v_inf;
}

static void orc_normalize(int64_t n3, double a, double* psi) {
  double s0 = 0.0;
  for (int64_t s = 0; s < n3; ++s) s0 += psi[s] * psi[s];
  const double f = 1.0 / sqrt(s0 * a * a * a);
  for (int64_t s = 0; s < n3; ++s) psi[s] *= f;
}

/* Excited states by projection (Sec. III, the snapshot method): remove from
 * psi its components along n states phi_k (each N^3 values, consecutive in
 * `states`), one after the other in the given order:
 *     psi <- psi - phi_k <phi_k|psi> / <phi_k|phi_k>.
 * With phi_0 the converged ground state and psi a snapshot, this is the
 * paper's estimate of the first excited state.  coef (optional) receives the
 * n coefficients <phi_k|psi>/<phi_k|phi_k>, each taken from psi as it stands
 * when phi_k is removed.  Sums are serial in lattice order. */
void orc_project_out(int64_t n3, const double* states, int n, double* psi, double* coef) {
  for (int k = 0; k < n; ++k) {
    const double* phi = states + (size_t)k * (size_t)n3;
    double pp = 0.0, pq = 0.0;
    for (int64_t s = 0; s < n3; ++s) {
      pp += phi[s] * phi[s];
      pq += phi[s] * psi[s];
    }
    const double c = pq / pp;
    if (coef) coef[k] = c;
    for (int64_t s = 0; s < n3; ++s) psi[s] -= c * phi[s];
  }
}

/* Imaginary-time evolution loop.  Step t (t = 0, 1, ...) maps psi_t to
 * psi_{t+1}; after every renorm_every-th step the state is rescaled to
 * a^3 sum psi^2 = 1 (Sec. III: renormalisation against underflow).  The
 * convergence test (Sec. V) looks at the state entering every check_every-th
 * step (t + 1 a multiple of check_every): it stops after that step when the
 * energy moved by at most rel_tol * |E - v_inf| since the previous check.
 * e_hist (optional, length max_steps / check_every) receives the checked
 * energies.  Returns the number of steps done; psi holds the final state. */
int64_t orc_evolve_deflated(int N, double L, double mass, double dt, const double* V,
                            double* psi, int64_t max_steps, int renorm_every, int check_every,
                            double rel_tol, double v_inf, int* converged, double* e_hist,
                            const double* states, int nstates, int project_every);

int64_t orc_evolve(int N, double L, double mass, double dt, const double* V, double* psi,
                   int64_t max_steps, int renorm_every, int check_every, double rel_tol,
                   double v_inf, int* converged, double* e_hist) {
  return orc_evolve_deflated(N, L, mass, dt, V, psi, max_steps, renorm_every, check_every,
                             rel_tol, v_inf, converged, e_hist, NULL, 0, 0);
}

/* The same loop relaxing to the lowest state orthogonal to n given states:
 * after every project_every-th step the state is projected against them
 * (orc_project_out), before the renormalisation of that step.  project_every
 * = 0 or nstates = 0: the plain loop. */
int64_t orc_evolve_deflated(int N, double L, double mass, double dt, const double* V,
                            double* psi, int64_t max_steps, int renorm_every, int check_every,
                            double rel_tol, double v_inf, int* converged, double* e_hist,
                            const double* states, int nstates, int project_every) {
  const double a = L / (double)N;
  const int64_t n3 = (int64_t)N * N * N;
  double* tmp = (double*)malloc((size_t)n3 * sizeof(double));
  if (!tmp) return -1;
  double e_prev = NAN;
  int64_t nchk = 0;
  *converged = 0;
  int64_t t = 0;
  while (t < max_steps) {
    const int check = check_every > 0 && ((t + 1) % check_every) == 0;
    double e_now = NAN;
    if (check) {
      double ob[6];
      orc_observables(N, L, mass, V, psi, v_inf, ob);
      e_now = ob[1];
      if (e_hist) e_hist[nchk] = e_now;
      ++nchk;
    }
    orc_step(N, L, mass, dt, V, psi, tmp);
    memcpy(psi, tmp, (size_t)n3 * sizeof(double));
    if (nstates > 0 && project_every > 0 && ((t + 1) % project_every) == 0)
      orc_project_out(n3, states, nstates, psi, NULL);
    if (renorm_every > 0 && ((t + 1) % renorm_every) == 0) orc_normalize(n3, a, psi);
    ++t;
    if (check) {
      if (!isnan(e_prev) && fabs(e_now - e_prev) <= rel_tol * fabs(e_now - v_inf)) {
        *converged = 1;
        break;
      }
      e_prev = e_now;
    }
  }
  free(tmp);
  return t;
}

/* Multi-resolution reseeding (Sec. VI, Sec. VII.G): the coarse state is
 * spread onto a finer lattice of the same box by trilinear interpolation.
 * Fine site j sits at x_j; in coarse index units it is t = x_j / a_c +
 * (N_c - 1)/2; with i0 = floor(t), w = t - i0 the 1-d weights are (1 - w) on
 * i0 and w on i0 + 1, coarse ghosts being zero.  The result is renormalised
 * to a_f^3 sum psi^2 = 1. */
void orc_upsample(int Nc, double L, const double* pc, int Nf, double* pf) {
  const double ac = L / (double)Nc, af = L / (double)Nf;
  int i0[3];
  double w[3];
#pragma omp parallel for schedule(static) private(i0, w)
  for (int jx = 0; jx < Nf; ++jx)
    for (int jy = 0; jy < Nf; ++jy)
      for (int jz = 0; jz < Nf; ++jz) {
        const int j[3] = {jx, jy, jz};
        for (int d = 0; d < 3; ++d) {
          const double t = orc_coord(j[d], Nf, af) / ac + 0.5 * (double)(Nc - 1);
          i0[d] = (int)floor(t);
          w[d] = t - (double)i0[d];
        }
        double v = 0.0;
        for (int cx = 0; cx < 2; ++cx)
          for (int cy = 0; cy < 2; ++cy)
            for (int cz = 0; cz < 2; ++cz) {
              const double wt = (cx ? w[0] : 1.0 - w[0]) * (cy ? w[1] : 1.0 - w[1]) *
                                (cz ? w[2] : 1.0 - w[2]);
              v += wt * orc_at(pc, Nc, i0[0] + cx, i0[1] + cy, i0[2] + cz);
            }
        pf[ORC_IDX(Nf, jx, jy, jz)] = v;
      }
  orc_normalize((int64_t)Nf * Nf * Nf, af, pf);
}

/* Gradient of E[psi_T] with respect to the potential field V, where psi_T is
 * obtained from psi_0 (held fixed) by T steps of Eq. (updateeq), each followed
 * by renormalisation.  Written as reverse-mode differentiation of that loop:
 *   M(V) psi = A psi + (B dt/2m) lap psi with A, B from V site by site;
 *   dA/dV = -dt B^2, dB/dV = -(dt/2) B^2, hence
 *   d(M psi)_i/dV_i = -(dt/2) B_i (psi_i + (M psi)_i);
 *   E = <psi|H|psi>/<psi|psi> gives dE/dpsi = 2 (H psi - E psi)/<psi|psi> and
 *   dE/dV_i (explicit) = psi_i^2 / <psi|psi>.
 * Because E is invariant under rescaling of psi, a renormalisation
 * psi_{t+1} = M psi_t / n_t only divides the adjoint by n_t.  The adjoint of
 * M is  (M^T l)_j = alpha_j l_j + sum_{i nbr of j} beta_i l_i  with
 * alpha = A - 6 B dt/(2 m a^2), beta = B dt / (2 m a^2).
 * All T + 1 states are stored (small lattices only).  G receives dE/dV
 * per site; returns E_T, or NAN on allocation failure. */
double orc_energy_grad_v(int N, double L, double mass, double dt, const double* V,
                         const double* psi0, int T, double* G) {
  const double a = L / (double)N;
  const double c = dt / (2.0 * mass * a * a);
  const int64_t n3 = (int64_t)N * N * N;
  double* states = (double*)malloc((size_t)(T + 1) * n3 * sizeof(double));
  double* norms = (double*)malloc((size_t)(T > 0 ? T : 1) * sizeof(double));
  double* lam = (double*)malloc((size_t)n3 * sizeof(double));
  double* lam2 = (double*)malloc((size_t)n3 * sizeof(double));
  double* hp = (double*)malloc((size_t)n3 * sizeof(double));
  if (!states || !norms || !lam || !lam2 || !hp) {
    free(states); free(norms); free(lam); free(lam2); free(hp);
    return NAN;
  }
  memcpy(states, psi0, (size_t)n3 * sizeof(double));
  for (int t = 0; t < T; ++t) { /* forward, keeping M psi_t / n_t and n_t */
    double* nxt = states + (size_t)(t + 1) * n3;
    orc_step(N, L, mass, dt, V, states + (size_t)t * n3, nxt);
    double s = 0.0;
    for (int64_t i = 0; i < n3; ++i) s += nxt[i] * nxt[i];
    norms[t] = sqrt(s);
    for (int64_t i = 0; i < n3; ++i) nxt[i] /= norms[t];
  }
  const double* pT = states + (size_t)T * n3;
  orc_hpsi(N, L, mass, V, pT, hp);
  double s0 = 0.0, eh = 0.0;
  for (int64_t i = 0; i < n3; ++i) { s0 += pT[i] * pT[i]; eh += pT[i] * hp[i]; }
  const double E = eh / s0;
  for (int64_t i = 0; i < n3; ++i) {
    lam[i] = 2.0 * (hp[i] - E * pT[i]) / s0;
    G[i] = pT[i] * pT[i] / s0;
  }
  for (int t = T - 1; t >= 0; --t) {
    const double* pt = states + (size_t)t * n3;
    const double* pn = states + (size_t)(t + 1) * n3; /* = M pt / n_t */
    for (int ix = 0; ix < N; ++ix)
      for (int iy = 0; iy < N; ++iy)
        for (int iz = 0; iz < N; ++iz) {
          const int64_t s = ORC_IDX(N, ix, iy, iz);
          const double B = 1.0 / (1.0 + 0.5 * dt * V[s]);
          /* V-derivative of step t at site s, through A and B of that site */
          G[s] += lam[s] * (-0.5 * dt * B) * (pt[s] + norms[t] * pn[s]) / norms[t];
        }
    for (int ix = 0; ix < N; ++ix)
      for (int iy = 0; iy < N; ++iy)
        for (int iz = 0; iz < N; ++iz) {
          const int64_t s = ORC_IDX(N, ix, iy, iz);
          const double B = 1.0 / (1.0 + 0.5 * dt * V[s]);
          const double A = (1.0 - 0.5 * dt * V[s]) / (1.0 + 0.5 * dt * V[s]);
          double acc = (A - 6.0 * B * c) * lam[s];
          const int nb[6][3] = {{ix - 1, iy, iz}, {ix + 1, iy, iz}, {ix, iy - 1, iz},
                                {ix, iy + 1, iz}, {ix, iy, iz - 1}, {ix, iy, iz + 1}};
          for (int k = 0; k < 6; ++k) {
            const int x = nb[k][0], y = nb[k][1], z = nb[k][2];
            if (x < 0 || y < 0 || z < 0 || x >= N || y >= N || z >= N) continue;
            const int64_t q = ORC_IDX(N, x, y, z);
            acc += (1.0 / (1.0 + 0.5 * dt * V[q])) * c * lam[q];
          }
          lam2[s] = acc / norms[t];
        }
    memcpy(lam, lam2, (size_t)n3 * sizeof(double));
  }
  free(states); free(norms); free(lam); free(lam2); free(hp);
  return E;
}

/* Derivative dV/dp[j] of the analytic potential of kind `kind`, as
 * orc_potential evaluates it, at every site (the Sec. VII potentials and the
 * Gaussian wells):
 *   CONST        dV/dp0 = 1;
 *   HO           dV/dp_d = p_d x_d^2 (x_0 = x, x_1 = y, x_2 = z);
 *   COULOMB      dV/dp0 = -1/r;
 *   COULOMB_REG  dV/dp0 = 1/a - 1/r for r >= a, 0 inside r < a;
 *   CORNELL      dV/dp0 = -1/r, dV/dp1 = r, dV/dp2 = z^2;
 *   WELLS        the oscillator part as HO for j < 3; for well k, with
 *                e = exp(-d^2 / (2 s^2)) and d the distance to its centre c,
 *                dV/dA = -e, dV/dc_d = -A e (x_d - c_d) / s^2,
 *                dV/ds = -A e d^2 / s^3;
 *   DODECA       dV/dp0 = 1 inside the solid, 0 outside.
 * Returns -1 for a parameter the kind does not have. */
int orc_potential_dv(int kind, const double* p, int np, int N, double L, int j, double* out) {
  const double a = L / (double)N;
  if (N < 1 || j < 0 || j >= np) return -1;
  switch (kind) {
    case ORC_POT_CONST: case ORC_POT_COULOMB: case ORC_POT_COULOMB_REG: case ORC_POT_DODECA:
      if (j != 0) return -1;
      break;
    case ORC_POT_HO: case ORC_POT_CORNELL:
      if (np < 3 || j > 2) return -1;
      break;
    case ORC_POT_WELLS:
      if (np < 3 || (np - 3) % 5 != 0) return -1;
      break;
    default: return -1;
  }
  const double half = 0.5 * (double)(N - 1) * a;
  for (int ix = 0; ix < N; ++ix)
    for (int iy = 0; iy < N; ++iy)
      for (int iz = 0; iz < N; ++iz) {
        const double xs[3] = {orc_coord(ix, N, a), orc_coord(iy, N, a), orc_coord(iz, N, a)};
        const double r = sqrt(xs[0] * xs[0] + xs[1] * xs[1] + xs[2] * xs[2]);
        double d = 0.0;
        switch (kind) {
          case ORC_POT_CONST: d = 1.0; break;
          case ORC_POT_HO: d = p[j] * xs[j] * xs[j]; break;
          case ORC_POT_COULOMB: d = -1.0 / r; break;
          case ORC_POT_COULOMB_REG: d = (r < a) ? 0.0 : (1.0 / a - 1.0 / r); break;
          case ORC_POT_CORNELL: d = (j == 0) ? -1.0 / r : (j == 1 ? r : xs[2] * xs[2]); break;
          case ORC_POT_WELLS:
            if (j < 3) {
              d = p[j] * xs[j] * xs[j];
            } else {
              const double* w = p + 3 + 5 * ((j - 3) / 5);
              const int q = (j - 3) % 5;
              const double dx = xs[0] - w[1], dy = xs[1] - w[2], dz = xs[2] - w[3];
              const double d2 = dx * dx + dy * dy + dz * dz;
              const double e = exp(-d2 / (2.0 * w[4] * w[4]));
              if (q == 0) d = -e;
              else if (q == 4) d = -w[0] * e * d2 / (w[4] * w[4] * w[4]);
              else d = -w[0] * e * (xs[q - 1] - w[q]) / (w[4] * w[4]);
            }
            break;
          case ORC_POT_DODECA:
            d = (N > 1 && orc_dodeca_inside(xs[0] / half, xs[1] / half, xs[2] / half)) ? 1.0 : 0.0;
            break;
        }
        out[ORC_IDX(N, ix, iy, iz)] = d;
      }
  return 0;
}

/* The Gaussian-well derivatives for the amplitudes A_k (j = 3 + 5k) and widths
 * s_k (j = 7 + 5k) only; -1 for any other j. */
int orc_wells_dv(const double* p, int np, int N, double L, int j, double* out) {
  if (np < 8 || (np - 3) % 5 != 0 || j < 3 || j >= np) return -1;
  const int r = (j - 3) % 5;
  if (r != 0 && r != 4) return -1;
  return orc_potential_dv(ORC_POT_WELLS, p, np, N, L, j, out);
}

/* Number of OpenMP threads the sweeps use (1 when built without OpenMP). */
int orc_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Set the number of OpenMP threads of later sweeps (for timing the oracle at
 * one thread and at all cores); no effect without OpenMP. */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  extern void omp_set_num_threads(int);
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
