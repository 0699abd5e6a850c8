/*
 * Reference oracle for the D3Q19 two-relaxation-time lattice Boltzmann
 * update with bounce-back walls and a constant body force.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU library; it has its own velocity
 * table and its own arithmetic, written as plainly as possible: scalar
 * double-precision loops, a collide pass followed by a separate stream pass
 * (the textbook two-step form that the paper lists among propagation
 * schemes not in its suite, Sect. 3, "Not Considered Propagation Steps").
 *
 * What it computes (the paper, Sect. 2, names the model and leaves its
 * formulas to the cited literature; the readings used here are):
 *   - D3Q19 velocity set: rest, 6 axis links (weight 1/18), 12 face
 *     diagonals (weight 1/36), rest weight 1/3, c_s^2 = 1/3.
 *     Canonical order: 0 rest; 1..6 = +x,-x,+y,-y,+z,-z; 7..18 = the
 *     diagonals in opposite pairs (xy, xz, yz planes).
 *   - TRT collision (Sect. 2): symmetric and antisymmetric halves of the
 *     populations relax with rates 1/tau+ and 1/tau-, with
 *     tau- = 1/2 + Lambda / (tau+ - 1/2).
 *   - Constant body force (Sect. 2.1) as a force density g, added with the
 *     second-order split-forcing term, split into its symmetric and
 *     antisymmetric halves; the velocity in the equilibrium and in the
 *     forcing term is u = (sum_i c_i f_i + g/2) / rho.
 *   - Bounce-back (Sect. 2 and Sect. 3.2): full-way (solid nodes store the
 *     arriving populations and send them back reversed one step later) or
 *     half-way (a population streaming into a solid node is reflected into
 *     the opposite direction of the node it left, in the same step).
 *   - Periodicity (Sect. 3.2) per axis: ora_run wraps every axis (a
 *     3-torus; walls are solid nodes of the mask, as the Sect. 2 geometries
 *     include their wall layers).  ora_run_box takes a bit mask of the axes
 *     that wrap; beyond the faces of the other axes every node counts as
 *     solid.  Under half-way bounce-back a population that would leave the
 *     box there is reflected like one aimed at a solid node.  Full-way
 *     bounce-back keeps reflected populations inside solid nodes, so it
 *     requires solid boundary layers on those axes and then wraps them
 *     (only solid nodes exchange populations across such a face).
 *
 * Threads: the two passes carry OpenMP "parallel for" pragmas over nodes
 * (collide) and over z planes (stream).  A plain build ignores them; the
 * OpenMP build is used only to time the oracle on all host cores.  Each
 * node's arithmetic, and each slot's single writer, is the same in both
 * builds, so their results are identical bit for bit.
 *
 * State layout: canonical pre-collision populations f[node][19] in double
 * precision, node = x + nx*(y + ny*z).  With half-way bounce-back solid
 * nodes carry no state and are kept at zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORA_Q 19

/* Velocity table written out by hand (see header comment for the order). */
static const int ORA_C[ORA_Q][3] = {
    {0, 0, 0},
    {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
    {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},
    {1, 0, 1},   {-1, 0, -1}, {1, 0, -1},  {-1, 0, 1},
    {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1},
};

static double ora_weight_of(int i) {
  int n2 = ORA_C[i][0] * ORA_C[i][0] + ORA_C[i][1] * ORA_C[i][1] +
           ORA_C[i][2] * ORA_C[i][2];
  if (n2 == 0) return 1.0 / 3.0;
  if (n2 == 1) return 1.0 / 18.0;
  return 1.0 / 36.0;
}

/* Opposite direction: the j with c_j = -c_i, found by search. */
static int ora_opposite_of(int i) {
  for (int j = 0; j < ORA_Q; ++j) {
    if (ORA_C[j][0] == -ORA_C[i][0] && ORA_C[j][1] == -ORA_C[i][1] &&
        ORA_C[j][2] == -ORA_C[i][2])
      return j;
  }
  return -1;
}

/* Weights and opposites, filled once from the two functions above. */
static double ORA_W[ORA_Q];
static int ORA_OPP[ORA_Q];
static int ora_tables_ready = 0;

static void ora_tables(void) {
  if (ora_tables_ready) return;
  for (int i = 0; i < ORA_Q; ++i) {
    ORA_W[i] = ora_weight_of(i);
    ORA_OPP[i] = ora_opposite_of(i);
  }
  ora_tables_ready = 1;
}

static double ora_weight(int i) { return ORA_W[i]; }
static int ora_opposite(int i) { return ORA_OPP[i]; }

/* Export the table: c[19][3], w[19], opp[19]. */
void ora_table(int* c, double* w, int* opp) {
  ora_tables();
  for (int i = 0; i < ORA_Q; ++i) {
    for (int a = 0; a < 3; ++a) c[3 * i + a] = ORA_C[i][a];
    w[i] = ora_weight(i);
    opp[i] = ora_opposite(i);
  }
}

/* Second-order equilibrium e_i = w_i rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u]. */
void ora_equilibrium(double rho, const double* u, double* e) {
  ora_tables();
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < ORA_Q; ++i) {
    double cu = ORA_C[i][0] * u[0] + ORA_C[i][1] * u[1] + ORA_C[i][2] * u[2];
    e[i] = ora_weight(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
  }
}

/* Density and force-shifted velocity u = (sum c f + g/2)/rho of one node. */
void ora_moments(const double* f, const double* g, double* rho_out,
                 double* u_out) {
  double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
  for (int i = 0; i < ORA_Q; ++i) {
    rho += f[i];
    for (int a = 0; a < 3; ++a) j[a] += ORA_C[i][a] * f[i];
  }
  *rho_out = rho;
  for (int a = 0; a < 3; ++a) u_out[a] = (j[a] + 0.5 * g[a]) / rho;
}

/* Forcing term F_i = w_i [3 (c_i - u) + 9 (c_i.u) c_i] . g */
static void ora_force_term(const double* u, const double* g, double* F) {
  for (int i = 0; i < ORA_Q; ++i) {
    double cu = ORA_C[i][0] * u[0] + ORA_C[i][1] * u[1] + ORA_C[i][2] * u[2];
    double s = 0.0;
    for (int a = 0; a < 3; ++a)
      s += (3.0 * (ORA_C[i][a] - u[a]) + 9.0 * cu * ORA_C[i][a]) * g[a];
    F[i] = ora_weight(i) * s;
  }
}

/* tau- from tau+ and the magic parameter Lambda = (tau+ - 1/2)(tau- - 1/2). */
double ora_tau_minus(double tau_plus, double magic) {
  return 0.5 + magic / (tau_plus - 0.5);
}

/* TRT collision with split forcing at one fluid node: f -> fstar. */
void ora_collide_node(const double* f, const double* g, double tau_plus,
                      double magic, double* fstar) {
  ora_tables();
  double rho, u[3], e[ORA_Q], F[ORA_Q];
  double lp = 1.0 / tau_plus;
  double lm = 1.0 / ora_tau_minus(tau_plus, magic);
  ora_moments(f, g, &rho, u);
  ora_equilibrium(rho, u, e);
  ora_force_term(u, g, F);
  for (int i = 0; i < ORA_Q; ++i) {
    int o = ora_opposite(i);
    double fp = 0.5 * (f[i] + f[o]), fm = 0.5 * (f[i] - f[o]);
    double ep = 0.5 * (e[i] + e[o]), em = 0.5 * (e[i] - e[o]);
    double Fp = 0.5 * (F[i] + F[o]), Fm = 0.5 * (F[i] - F[o]);
    fstar[i] = f[i] - lp * (fp - ep) - lm * (fm - em) + (1.0 - 0.5 * lp) * Fp +
               (1.0 - 0.5 * lm) * Fm;
  }
}

static int64_t ora_wrap(int64_t v, int64_t n) {
  v %= n;
  return v < 0 ? v + n : v;
}

static int64_t ora_node(int64_t x, int64_t y, int64_t z, int nx, int ny,
                        int nz) {
  return ora_wrap(x, nx) + (int64_t)nx * (ora_wrap(y, ny) + (int64_t)ny * ora_wrap(z, nz));
}

/* 1 if coordinate v of an axis of n nodes lies outside the box and the
   axis does not wrap (its bit in `periodic` is clear). */
static int ora_outside(int64_t v, int n, unsigned periodic, int axis) {
  return !((periodic >> axis) & 1u) && (v < 0 || v >= n);
}

/* 1 if every node of the two boundary layers of each non-wrapping axis is
   solid. */
static int ora_faces_solid(int nx, int ny, int nz, const uint8_t* mask,
                           unsigned periodic) {
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        int on_face = (!(periodic & 1u) && (x == 0 || x == nx - 1)) ||
                      (!(periodic & 2u) && (y == 0 || y == ny - 1)) ||
                      (!(periodic & 4u) && (z == 0 || z == nz - 1));
        if (on_face && mask[ora_node(x, y, z, nx, ny, nz)] == 0) return 0;
      }
  return 1;
}

/*
 * Advance the canonical state f[N][19] by nsteps (collide, then stream).
 * bounce: 0 = full-way, 1 = half-way.  periodic: bit 0 x, 1 y, 2 z set for
 * the axes that wrap.  Returns 0, or -1 on bad arguments (including
 * full-way with a fluid node on a wall face) or allocation failure.
 */
int ora_run_box(int nx, int ny, int nz, unsigned periodic, const uint8_t* mask,
                int bounce, double tau_plus, double magic, const double* g,
                double* f, int nsteps) {
  ora_tables();
  if (nx < 1 || ny < 1 || nz < 1 || !mask || !f || !g || nsteps < 0) return -1;
  if (!(tau_plus > 0.5) || !(magic > 0.0) || (bounce != 0 && bounce != 1)) return -1;
  if (periodic > 7u) return -1;
  if (bounce == 0 && !ora_faces_solid(nx, ny, nz, mask, periodic)) return -1;
  int64_t n_nodes = (int64_t)nx * ny * nz;
  double* post = (double*)malloc(sizeof(double) * ORA_Q * n_nodes);
  if (!post) return -1;
  for (int step = 0; step < nsteps; ++step) {
    /* collide (the OpenMP build splits the nodes over threads; every
       node's arithmetic is the same in either build) */
#pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < n_nodes; ++n) {
      const double* fn = f + ORA_Q * n;
      double* pn = post + ORA_Q * n;
      if (mask[n] == 0) {
        ora_collide_node(fn, g, tau_plus, magic, pn);
      } else if (bounce == 0) {
        for (int i = 0; i < ORA_Q; ++i) pn[i] = fn[ora_opposite(i)];
      } else {
        for (int i = 0; i < ORA_Q; ++i) pn[i] = 0.0;
      }
    }
    /* stream */
    if (bounce == 1) memset(f, 0, sizeof(double) * ORA_Q * n_nodes);
    /* each target slot has one writer: f(x + c_i, i) from x, or, for a
       solid target (or one beyond a wall face) under half-way bounce-back,
       f(x, opp i) from x itself */
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          int64_t n = ora_node(x, y, z, nx, ny, nz);
          if (bounce == 1 && mask[n] != 0) continue;
          for (int i = 0; i < ORA_Q; ++i) {
            int64_t tx = x + ORA_C[i][0], ty = y + ORA_C[i][1], tz = z + ORA_C[i][2];
            int beyond = ora_outside(tx, nx, periodic, 0) ||
                         ora_outside(ty, ny, periodic, 1) ||
                         ora_outside(tz, nz, periodic, 2);
            int64_t t = ora_node(tx, ty, tz, nx, ny, nz);
            if (bounce == 0 || (!beyond && mask[t] == 0))
              f[ORA_Q * t + i] = post[ORA_Q * n + i];
            else
              f[ORA_Q * n + ora_opposite(i)] = post[ORA_Q * n + i];
          }
        }
  }
  free(post);
  return 0;
}

/* ora_run_box with every axis wrapping. */
int ora_run(int nx, int ny, int nz, const uint8_t* mask, int bounce,
            double tau_plus, double magic, const double* g, double* f,
            int nsteps) {
  return ora_run_box(nx, ny, nz, 7u, mask, bounce, tau_plus, magic, g, f, nsteps);
}

/* Density and velocity fields of the canonical state; solids report 0. */
void ora_macroscopic(int64_t n_nodes, const uint8_t* mask, const double* f,
                     const double* g, double* rho, double* u /* [N][3] */) {
  for (int64_t n = 0; n < n_nodes; ++n) {
    if (mask[n] != 0) {
      rho[n] = 0.0;
      u[3 * n] = u[3 * n + 1] = u[3 * n + 2] = 0.0;
      continue;
    }
    ora_moments(f + ORA_Q * n, g, rho + n, u + 3 * n);
  }
}

/* Rest state f_i = w_i on fluid nodes (and on solids for full-way). */
void ora_rest_state(int64_t n_nodes, const uint8_t* mask, int bounce,
                    double* f) {
  ora_tables();
  for (int64_t n = 0; n < n_nodes; ++n)
    for (int i = 0; i < ORA_Q; ++i)
      f[ORA_Q * n + i] = (bounce == 1 && mask[n] != 0) ? 0.0 : ora_weight(i);
}
