/*
 * rt_oracle.c -- plain, slow FP64 CPU oracle for Monte-Carlo line-by-line
 * ray tracing through finite volumes (Collange, Daumas, Defour,
 * "Graphic processors to speed-up simulations for the design of high
 * performance solar receptors", Section 3, Eqs. (1)-(4)).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or constant table
 * with the HIP library: every formula below is written out from the paper's
 * equations and from the readings recorded in the design notes.
 *
 * Precision: IEEE binary64 throughout, libm exp/expm1/pow, no fast-math,
 * no FMA contraction (built with -ffp-contract=off).  Loops follow the
 * definition's own index order; the only parallelism is an OpenMP loop over
 * independent cells in the absorption-coefficient and Planck tables, which
 * leaves every per-element summation order unchanged.
 *
 * Parity pins (tests/test_oracle_*.py):
 *   philox     numpy.random.Philox raw words (bit-exact)
 *   rays       face uniformity, in-face uniformity, cosine-law moments
 *   traversal  brute-force rational plane-crossing enumeration, Cauchy chord
 *   kappa      Poisson-comb closed form of a periodic Lorentz sum, windowed
 *              integral (2/pi) atan(cutoff/gamma), T = T_ref gives ratio 1
 *   planck     Stefan-Boltzmann integral, Wien and Rayleigh-Jeans limits
 *   march      slab transmissivity, kappa = 0 pass-through, thick limit,
 *              per-ray energy balance
 *   adaptive   vanishing tolerance gives the plain sum; one isolated line
 *              keeps exactly the points where its plain value reaches the
 *              threshold; nesting in the tolerance; the dropped remainder
 *              within its bound; brute-force value-criterion counts
 *   wing return  nothing to return at vanishing tolerance; one isolated
 *              line dropped whole returns its Poisson-comb band mean; the
 *              band integral of the plain sum within the midpoint rule's
 *              bound; a symmetric line's two wings in closed form
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __int128 i128;

/* ---- physical constants: SI 2019 exact values ------------------------- */
static const double ORC_H = 6.62607015e-34;  /* Planck constant, J s      */
static const double ORC_C = 299792458.0;     /* speed of light, m/s       */
static const double ORC_KB = 1.380649e-23;   /* Boltzmann constant, J/K   */
static const double ORC_ATM = 101325.0;      /* 1 atm in Pa               */

/* second radiation constant c2 = h c / k_B, in cm K */
static double orc_c2(void) { return ORC_H * ORC_C / ORC_KB * 100.0; }
/* first radiation constant for radiance per wavenumber in cm^-1:
 * 2 h c^2 [W m^2] times (100 cm^-1 per m^-1)^4 / (100 per cm^-1 bin)
 * -> W m^-2 sr^-1 (cm^-1)^-1 with nu in cm^-1 */
static double orc_c1(void) { return 2.0 * ORC_H * ORC_C * ORC_C * 1e8; }

double orc_const_c1(void) { return orc_c1(); }
double orc_const_c2(void) { return orc_c2(); }

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* threads of the OpenMP loops over cells (timing on one core or all) */
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n >= 1) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* ======================================================================
 * Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11), written from its published definition: ten
 * rounds of two 64x64->128 multiplications by the round multipliers, the
 * high halves xored with the other counter words and the key, followed by
 * a Weyl-sequence key bump between rounds.
 * ==================================================================== */
void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2],
                       uint64_t out[4]) {
  const uint64_t mult0 = 0xD2E7470EE14C6C93ULL, mult1 = 0xCA5A826395121157ULL;
  const uint64_t weyl0 = 0x9E3779B97F4A7C15ULL, weyl1 = 0xBB67AE8584CAA73BULL;
  uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
  uint64_t k0 = key_in[0], k1 = key_in[1];
  for (int round = 0; round < 10; ++round) {
    unsigned __int128 p0 = (unsigned __int128)mult0 * x0;
    unsigned __int128 p1 = (unsigned __int128)mult1 * x2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ x1 ^ k0;
    uint64_t n1 = lo1;
    uint64_t n2 = hi0 ^ x3 ^ k1;
    uint64_t n3 = lo0;
    x0 = n0; x1 = n1; x2 = n2; x3 = n3;
    k0 += weyl0; k1 += weyl1;
  }
  out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* floor(w * m / 2^64): an integer uniform on [0, m) when w is uniform */
static uint64_t orc_mulhi(uint64_t w, uint64_t m) {
  return (uint64_t)(((unsigned __int128)w * m) >> 64);
}

/* floor(sqrt(v)) for 0 <= v < 2^62, by bisection on exact integers */
static int64_t orc_isqrt(int64_t v) {
  int64_t lo = 0, hi = 1;
  while (hi * hi <= v) hi *= 2;
  /* invariant lo^2 <= v < hi^2 */
  while (hi - lo > 1) {
    int64_t mid = lo + (hi - lo) / 2;
    if (mid * mid <= v) lo = mid; else hi = mid;
  }
  return lo;
}

/* ======================================================================
 * Ray sampling (the paper averages the effect of individual Monte-Carlo
 * rays, Section 3; it fixes no sampling law).  Reading used here: a point
 * uniform on the boundary surface and a cosine-weighted inward direction
 * (Malley's method: uniform point in the unit disk lifted to the
 * hemisphere), all in exact integer arithmetic so that traversal is
 * reproducible bit for bit.
 *
 * Fixed-point frame: one cell edge = 2^21 units.  In-face origin
 * coordinates are odd, so an origin never lies on a cell edge.
 * Direction components are integers of magnitude < 2^20 (+1).
 *
 * Words: key = (seed, 1), counter = (r, block, 0, 0).
 *   block 0: w0 -> face (area-weighted), w1, w2 -> in-face position,
 *            w3 -> first disk candidate; blocks 1..15 -> further
 *            candidates (4 per block).  Candidate word w gives
 *            A = (w & (2^21-1)) - 2^20, B = ((w >> 21) & (2^21-1)) - 2^20,
 *            accepted iff A^2 + B^2 < 2^40.  If all 61 candidates are
 *            rejected the ray goes along the inward normal (A = B = 0).
 *   normal component Cn = isqrt(2^40 - A^2 - B^2) >= 1.
 * Faces: f = 2*axis + side; side 0 is the low face (inward +), side 1 the
 * high face (inward -); tangent axes t1 = (axis+1)%3, t2 = (axis+2)%3.
 * ==================================================================== */
#define ORC_CELL_UNITS (1LL << 21)

int orc_ray(uint64_t seed, uint64_t r, int nx, int ny, int nz,
            int64_t O[3], int64_t D[3], int32_t* face_out) {
  const int64_t n[3] = {nx, ny, nz};
  const uint64_t key[2] = {seed, 1u};
  uint64_t ctr[4] = {r, 0u, 0u, 0u};
  uint64_t w[4];
  orc_philox4x64_10(ctr, key, w);

  /* area of each face in cell-face units, faces in the fixed order */
  uint64_t area[6];
  for (int f = 0; f < 6; ++f) {
    int a = f / 2;
    area[f] = (uint64_t)(n[(a + 1) % 3] * n[(a + 2) % 3]);
  }
  uint64_t total = 0;
  for (int f = 0; f < 6; ++f) total += area[f];
  uint64_t u = orc_mulhi(w[0], total);
  int face = 0;
  uint64_t acc = area[0];
  while (u >= acc) { ++face; acc += area[face]; }

  const int axis = face / 2, side = face % 2;
  const int t1 = (axis + 1) % 3, t2 = (axis + 2) % 3;
  O[axis] = side ? n[axis] * ORC_CELL_UNITS : 0;
  O[t1] = 2 * (int64_t)orc_mulhi(w[1], (uint64_t)n[t1] << 20) + 1;
  O[t2] = 2 * (int64_t)orc_mulhi(w[2], (uint64_t)n[t2] << 20) + 1;

  const int64_t R = 1LL << 20, R2 = R * R, M21 = (1LL << 21) - 1;
  int64_t A = 0, B = 0;
  int found = 0;
  for (int k = 0; k < 61 && !found; ++k) {
    uint64_t cand;
    if (k == 0) {
      cand = w[3];
    } else {
      int blk = 1 + (k - 1) / 4, pos = (k - 1) % 4;
      if (pos == 0) {
        ctr[1] = (uint64_t)blk;
        orc_philox4x64_10(ctr, key, w);
      }
      cand = w[pos];
    }
    int64_t a = (int64_t)(cand & (uint64_t)M21) - R;
    int64_t b = (int64_t)((cand >> 21) & (uint64_t)M21) - R;
    if (a * a + b * b < R2) { A = a; B = b; found = 1; }
  }
  int64_t Cn = orc_isqrt(R2 - A * A - B * B);
  D[axis] = side ? -Cn : Cn;
  D[t1] = A;
  D[t2] = B;
  if (face_out) *face_out = face;
  return 0;
}

/* ======================================================================
 * Traversal: the cells a straight ray crosses, in order, with the length
 * it spends inside each (the paper's volumes of length l, Eq. (3)).
 * Written as the plain definition: list every grid plane the ray meets
 * before leaving the box as an exact rational parameter t = num/den,
 * sort, merge equal parameters (several planes met at once: an edge or a
 * corner, crossed in one step, so cells touched only at an edge or corner
 * are not visited), and take each cell as the one containing the midpoint
 * of consecutive parameters.  All of it is exact 128-bit integer work; the
 * length (t_b - t_a) |D| h / 2^21 is converted to FP64 at the very end.
 * ==================================================================== */
typedef struct { i128 num, den; } orc_frac; /* den > 0 */

static int orc_frac_cmp(const void* pa, const void* pb) {
  const orc_frac* a = (const orc_frac*)pa;
  const orc_frac* b = (const orc_frac*)pb;
  i128 l = a->num * b->den, r = b->num * a->den;
  return (l < r) ? -1 : (l > r) ? 1 : 0;
}

static i128 orc_floor_div(i128 a, i128 b) { /* b > 0 */
  i128 q = a / b;
  if ((a % b != 0) && (a < 0)) q -= 1;
  return q;
}

int orc_segments(int nx, int ny, int nz, double h_cm, const int64_t O[3],
                 const int64_t D[3], int32_t* cells, double* len_cm,
                 int cap) {
  const int64_t n[3] = {nx, ny, nz};
  const i128 U = ORC_CELL_UNITS;
  /* exit parameter: the smallest t at which some coordinate reaches the
   * far boundary of the box along its direction */
  orc_frac t_exit = {0, 0};
  for (int k = 0; k < 3; ++k) {
    if (D[k] == 0) continue;
    i128 bound = (D[k] > 0) ? (i128)n[k] * U : 0;
    orc_frac t = {(bound - O[k]) * (D[k] > 0 ? 1 : -1), D[k] > 0 ? D[k] : -D[k]};
    if (t_exit.den == 0 || orc_frac_cmp(&t, &t_exit) < 0) t_exit = t;
  }
  if (t_exit.den == 0) return -1; /* zero direction */

  /* every plane p*U with t in (0, t_exit] */
  int64_t total_planes = n[0] + n[1] + n[2] + 3;
  orc_frac* ts = (orc_frac*)malloc(sizeof(orc_frac) * (size_t)total_planes);
  int nt = 0;
  for (int k = 0; k < 3; ++k) {
    if (D[k] == 0) continue;
    i128 den = D[k] > 0 ? D[k] : -D[k];
    for (int64_t p = 0; p <= n[k]; ++p) {
      i128 num = ((i128)p * U - O[k]) * (D[k] > 0 ? 1 : -1);
      orc_frac t = {num, den};
      if (num <= 0) continue;
      if (orc_frac_cmp(&t, &t_exit) > 0) continue;
      ts[nt++] = t;
    }
  }
  qsort(ts, (size_t)nt, sizeof(orc_frac), orc_frac_cmp);
  /* merge equal parameters */
  int m = 0;
  for (int i = 0; i < nt; ++i) {
    if (m > 0 && orc_frac_cmp(&ts[i], &ts[m - 1]) == 0) continue;
    ts[m++] = ts[i];
  }
  double dlen = sqrt((double)D[0] * (double)D[0] + (double)D[1] * (double)D[1] +
                     (double)D[2] * (double)D[2]);
  double unit_cm = h_cm / (double)ORC_CELL_UNITS;
  int count = 0;
  orc_frac ta = {0, 1};
  for (int i = 0; i < m; ++i) {
    orc_frac tb = ts[i];
    /* midpoint position along axis k: O_k + (ta + tb)/2 * D_k, as the
     * rational (2 O_k ta.den tb.den + (ta.num tb.den + tb.num ta.den) D_k)
     *            / (2 ta.den tb.den) */
    i128 den = 2 * ta.den * tb.den;
    i128 sum = ta.num * tb.den + tb.num * ta.den;
    int64_t idx[3];
    for (int k = 0; k < 3; ++k) {
      i128 pos = 2 * (i128)O[k] * ta.den * tb.den + sum * D[k];
      idx[k] = (int64_t)orc_floor_div(pos, den * U);
    }
    if (idx[0] < 0 || idx[0] >= n[0] || idx[1] < 0 || idx[1] >= n[1] ||
        idx[2] < 0 || idx[2] >= n[2]) {
      free(ts);
      return -2; /* cannot happen for an origin on the boundary */
    }
    if (count >= cap) { free(ts); return -3; }
    cells[count] = (int32_t)(idx[0] + n[0] * (idx[1] + n[1] * idx[2]));
    /* tb - ta = (tb.num ta.den - ta.num tb.den) / (ta.den tb.den), exact */
    i128 dnum = tb.num * ta.den - ta.num * tb.den;
    i128 dden = ta.den * tb.den;
    len_cm[count] = ((double)dnum / (double)dden) * dlen * unit_cm;
    ++count;
    ta = tb;
  }
  free(ts);
  return count;
}

/* ======================================================================
 * Gas state and line parameters.
 *   u_c = x_c p_c / (k_B T_c), molecules per cm^3 (ideal gas; the paper's
 *         u_g is the density of absorbing molecule), p in atm.
 *   Eq. (1): S(T)/S(T_ref) = Q(T_ref)/Q(T) * exp(-c2 E/T)/exp(-c2 E/T_ref)
 *            * (1 - exp(-c2 nu_i/T)) / (1 - exp(-c2 nu_i/T_ref)),
 *            with the partition-function ratio Q(T_ref)/Q(T) read as
 *            (T_ref/T)^1.5; ratio = 1 when no lower-state energies are
 *            given.
 *   half width gamma_ci = gamma_i (p_c / 1 atm) (T_ref/T_c)^n_i.
 *   Eq. (2) with a Lorentz profile f(d) = (gamma/pi)/(d^2 + gamma^2),
 *   hard cutoff |nu_j - nu_i| <= cutoff in grid units |j - r_i| <= K,
 *   r_i = (nu_i - nu_0)/dnu, K = cutoff/dnu:
 *   kappa_c(nu_j) = u_c * sum_i S_i ratio_ci gamma_ci
 *                       / (pi ((j - r_i)^2 dnu^2 + gamma_ci^2))   [cm^-1]
 * ==================================================================== */
double orc_density(double T, double x, double p_atm) {
  return x * p_atm * ORC_ATM / (ORC_KB * T) * 1e-6;
}

double orc_strength_ratio(double T, double T_ref, double nu_line,
                          double E_lower, int have_E) {
  if (!have_E) return 1.0;
  const double c2 = orc_c2();
  double q = pow(T_ref / T, 1.5);
  double boltz = exp(-c2 * E_lower / T) / exp(-c2 * E_lower / T_ref);
  /* 1 - exp(-y) evaluated as -expm1(-y): the same value, without the
   * cancellation of a literal subtraction for small y */
  double stim = expm1(-c2 * nu_line / T) / expm1(-c2 * nu_line / T_ref);
  return q * boltz * stim;
}

double orc_half_width(double gamma_ref, double n_T, double T, double T_ref,
                      double p_atm) {
  return gamma_ref * p_atm * pow(T_ref / T, n_T);
}

/* kappa rows for the listed cells: out[row][j], row = index into
 * cell_list.  Lines are taken in input order for every j. */
int orc_kappa(int n_cells_listed, const int32_t* cell_list, const double* T,
              const double* x, const double* p, int n_lines,
              const double* nu_line, const double* S_ref,
              const double* gamma_ref, const double* n_T,
              const double* E_lower /* NULL: ratio 1 */, double T_ref,
              double cutoff_cm, double nu0, double dnu, int n_nu,
              double* out) {
  double Kd = cutoff_cm / dnu;
  double K = floor(Kd + 0.5);
  if (fabs(Kd - K) > 1e-9 * (K > 1.0 ? K : 1.0)) return -1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int row = 0; row < n_cells_listed; ++row) {
    int c = cell_list[row];
    double* kap = out + (size_t)row * (size_t)n_nu;
    for (int j = 0; j < n_nu; ++j) kap[j] = 0.0;
    double u = orc_density(T[c], x[c], p[c]);
    for (int i = 0; i < n_lines; ++i) {
      double r = (nu_line[i] - nu0) / dnu;
      double s = orc_strength_ratio(T[c], T_ref, nu_line[i],
                                    E_lower ? E_lower[i] : 0.0, E_lower != NULL);
      double g = orc_half_width(gamma_ref[i], n_T[i], T[c], T_ref, p[c]);
      /* candidate j around the window, widened by one on each side; the
       * exact membership test j - K <= r <= j + K decides */
      double jlo_d = ceil(r - K) - 1.0, jhi_d = floor(r + K) + 1.0;
      if (jhi_d < 0.0 || jlo_d > (double)(n_nu - 1)) continue;
      long jlo = jlo_d < 0.0 ? 0 : (long)jlo_d;
      long jhi = jhi_d > (double)(n_nu - 1) ? n_nu - 1 : (long)jhi_d;
      for (long j = jlo; j <= jhi; ++j) {
        double jd = (double)j;
        if (!(jd - K <= r && r <= jd + K)) continue;
        double delta = (jd - r) * dnu;
        kap[j] += S_ref[i] * s * g / (M_PI * (delta * delta + g * g));
      }
    }
    for (int j = 0; j < n_nu; ++j) kap[j] *= u;
  }
  return 0;
}

/* The paper's own formulation of Eq. (2) (its Section 3 and listing): every
 * line contributes at the 16 grid points j = m - 7 .. m + 8, m = floor(r),
 * r = (nu - nu0)/dnu, with its Lorentz shape at the reference state
 * (gamma_ref, 1 atm) -- a profile the paper tabulates once per line --
 * scaled per cell by the density u and the Eq. (1) strength ratio s:
 * kappa_c(nu_j) = u_c sum_i S_i s_ci gamma_i / (pi ((j - r_i)^2 dnu^2 + gamma_i^2)).
 * There is no per-cell half width and no cutoff beyond the 16 points. */
int orc_kappa_table16(int n_cells_listed, const int32_t* cell_list, const double* T,
                      const double* x, const double* p, int n_lines,
                      const double* nu_line, const double* S_ref,
                      const double* gamma_ref, const double* E_lower /* NULL: ratio 1 */,
                      double T_ref, double nu0, double dnu, int n_nu, double* out) {
#pragma omp parallel for schedule(dynamic, 1)
  for (int row = 0; row < n_cells_listed; ++row) {
    int c = cell_list[row];
    double* kap = out + (size_t)row * (size_t)n_nu;
    for (int j = 0; j < n_nu; ++j) kap[j] = 0.0;
    double u = orc_density(T[c], x[c], p[c]);
    for (int i = 0; i < n_lines; ++i) {
      double r = (nu_line[i] - nu0) / dnu;
      double fm = floor(r);
      if (!(fabs(fm) < 4.0e15)) continue;
      long m = (long)fm;
      if (m + 8 < 0 || m - 7 > (long)(n_nu - 1)) continue;
      double s = orc_strength_ratio(T[c], T_ref, nu_line[i],
                                    E_lower ? E_lower[i] : 0.0, E_lower != NULL);
      double g = gamma_ref[i];
      for (long j = m - 7; j <= m + 8; ++j) {
        if (j < 0 || j > (long)(n_nu - 1)) continue;
        double delta = ((double)j - r) * dnu;
        kap[j] += S_ref[i] * s * g / (M_PI * (delta * delta + g * g));
      }
    }
    for (int j = 0; j < n_nu; ++j) kap[j] *= u;
  }
  return 0;
}

/* ======================================================================
 * Adaptive line windows: the paper's announced next version (its
 * conclusion), in which the number of points evaluated per line follows the
 * local temperature and the line's intensity.  Reading used here:
 *   - reference level of cell c: the band mean of its untruncated line sum,
 *     kbar_c = u_c sbar_c, sbar_c = sum_i S_i s_ci / (n_nu dnu), over the
 *     lines whose hard-cutoff window meets the grid;
 *   - line i keeps point j in cell c while its Lorentz value there is at
 *     least eps kbar_c: u S s g / (pi (D^2 + g^2)) >= eps u sbar, i.e.
 *     D^2 <= W2 = S s g / (pi eps sbar) - g^2 (u cancels), a half width of
 *     w_ci = sqrt(W2) / dnu grid points, none at all when W2 < 0;
 *   - the window is shared by each run of `group` consecutive cells
 *     (c / group): the widest w_ci of its cells, never beyond the hard
 *     cutoff K.  Every cell therefore keeps at least the points its own
 *     rule asks for;
 *   - point j is kept when it is in the hard window (the plain sum's exact
 *     test) and fabs(j - r_i) <= min(K, w), both in binary64.
 * When every line has zero strength (sbar = 0) the hard window is kept.
 * ==================================================================== */
static int orc_meets_grid(double r, double K, int n_nu) {
  return r >= -K && r <= (double)(n_nu - 1) + K;
}

double orc_mean_strength(double T, int n_lines, const double* nu_line, const double* S_ref,
                         const double* E_lower, double T_ref, double cutoff_cm, double nu0,
                         double dnu, int n_nu) {
  double K = floor(cutoff_cm / dnu + 0.5);
  double sum = 0.0;
  for (int i = 0; i < n_lines; ++i) {
    double r = (nu_line[i] - nu0) / dnu;
    if (!orc_meets_grid(r, K, n_nu)) continue;
    double s = orc_strength_ratio(T, T_ref, nu_line[i], E_lower ? E_lower[i] : 0.0,
                                  E_lower != NULL);
    sum += S_ref[i] * s;
  }
  return sum / ((double)n_nu * dnu);
}

/* w_ci in grid points, -1 when the line keeps no point in this cell */
static double orc_window_points(double T, double p, double sbar, int i, const double* nu_line,
                                const double* S_ref, const double* gamma_ref, const double* n_T,
                                const double* E_lower, double T_ref, double dnu, double eps,
                                double K) {
  if (sbar == 0.0) return K;
  double s = orc_strength_ratio(T, T_ref, nu_line[i], E_lower ? E_lower[i] : 0.0,
                                E_lower != NULL);
  double g = orc_half_width(gamma_ref[i], n_T[i], T, T_ref, p);
  double num = S_ref[i] * s * g;
  double den = M_PI * eps * sbar;
  double W2 = num / den - g * g;
  if (W2 < 0.0) return -1.0;
  return sqrt(W2) / dnu;
}

/* the group's shared half width of line i, min(K, max over its cells) */
static double orc_group_window(int grp, int group, int n_cells, const double* T,
                               const double* p, const double* sbar_grp, int i,
                               const double* nu_line, const double* S_ref,
                               const double* gamma_ref, const double* n_T,
                               const double* E_lower, double T_ref, double dnu, double eps,
                               double K) {
  double w = -1.0;
  for (int k = 0; k < group; ++k) {
    int c = grp * group + k;
    if (c >= n_cells) break;
    double wc = orc_window_points(T[c], p[c], sbar_grp[k], i, nu_line, S_ref, gamma_ref, n_T,
                                  E_lower, T_ref, dnu, eps, K);
    if (wc > w) w = wc;
  }
  return w < K ? w : K;
}

static int orc_kept(double jd, double r, double K, double hw) {
  return (jd - K <= r && r <= jd + K) && hw >= 0.0 && fabs(jd - r) <= hw;
}

/* kappa rows of the adaptive form for the listed cells (n_cells: the whole
 * grid, whose T, x, p are indexed by cell); lines in input order for every
 * j, as in orc_kappa.  Returns -1 on a non-integer cutoff/dnu, -2 on bad
 * eps or group. */
int orc_kappa_adaptive(int n_cells_listed, const int32_t* cell_list, int n_cells,
                       const double* T, const double* x, const double* p, int n_lines,
                       const double* nu_line, const double* S_ref, const double* gamma_ref,
                       const double* n_T, const double* E_lower, double T_ref,
                       double cutoff_cm, double nu0, double dnu, int n_nu, double eps,
                       int group, double* out) {
  double Kd = cutoff_cm / dnu;
  double K = floor(Kd + 0.5);
  if (fabs(Kd - K) > 1e-9 * (K > 1.0 ? K : 1.0)) return -1;
  if (!(eps > 0.0) || group < 1 || group > 64) return -2;
#pragma omp parallel for schedule(dynamic, 1)
  for (int row = 0; row < n_cells_listed; ++row) {
    int c = cell_list[row];
    int grp = c / group;
    double sbar[64];
    for (int k = 0; k < group; ++k) {
      int cc = grp * group + k;
      sbar[k] = cc < n_cells ? orc_mean_strength(T[cc], n_lines, nu_line, S_ref, E_lower,
                                                 T_ref, cutoff_cm, nu0, dnu, n_nu)
                             : 0.0;
    }
    double* kap = out + (size_t)row * (size_t)n_nu;
    for (int j = 0; j < n_nu; ++j) kap[j] = 0.0;
    double u = orc_density(T[c], x[c], p[c]);
    for (int i = 0; i < n_lines; ++i) {
      double r = (nu_line[i] - nu0) / dnu;
      if (!orc_meets_grid(r, K, n_nu)) continue;
      double hw = orc_group_window(grp, group, n_cells, T, p, sbar, i, nu_line, S_ref,
                                   gamma_ref, n_T, E_lower, T_ref, dnu, eps, K);
      if (hw < 0.0) continue;
      double s = orc_strength_ratio(T[c], T_ref, nu_line[i],
                                    E_lower ? E_lower[i] : 0.0, E_lower != NULL);
      double g = orc_half_width(gamma_ref[i], n_T[i], T[c], T_ref, p[c]);
      double jlo_d = ceil(r - K) - 1.0, jhi_d = floor(r + K) + 1.0;
      long jlo = jlo_d < 0.0 ? 0 : (long)jlo_d;
      long jhi = jhi_d > (double)(n_nu - 1) ? n_nu - 1 : (long)jhi_d;
      for (long j = jlo; j <= jhi; ++j) {
        double jd = (double)j;
        if (!orc_kept(jd, r, K, hw)) continue;
        double delta = (jd - r) * dnu;
        kap[j] += S_ref[i] * s * g / (M_PI * (delta * delta + g * g));
      }
    }
    for (int j = 0; j < n_nu; ++j) kap[j] *= u;
  }
  return 0;
}

/* Number of (cell, line, grid point) evaluations the adaptive form keeps
 * over the whole grid.  The kept points of a line are contiguous around its
 * centre (fabs(j - r) grows monotonically away from r, and the hard window
 * is an interval), so on each side of c0 = floor(r) the last kept offset is
 * found by bisection on the kept test itself; offsets beyond K + 1 are
 * never kept. */
static long orc_last_kept(double c0, int dir, double r, double K, double hw) {
  /* largest t >= t0 with c0 + dir t kept, t0 = 1 above and 0 below the
   * centre; t0 - 1 when none is */
  long t0 = dir > 0 ? 1 : 0;
  if (!orc_kept(c0 + dir * (double)t0, r, K, hw)) return t0 - 1;
  long lo = t0, hi = (long)K + 2;     /* kept at lo, not kept at hi */
  while (hi - lo > 1) {
    long mid = lo + (hi - lo) / 2;
    if (orc_kept(c0 + dir * (double)mid, r, K, hw)) lo = mid; else hi = mid;
  }
  return lo;
}

double orc_adaptive_evals(int n_cells, const double* T, const double* p, int n_lines,
                          const double* nu_line, const double* S_ref, const double* gamma_ref,
                          const double* n_T, const double* E_lower, double T_ref,
                          double cutoff_cm, double nu0, double dnu, int n_nu, double eps,
                          int group) {
  double Kd = cutoff_cm / dnu;
  double K = floor(Kd + 0.5);
  if (fabs(Kd - K) > 1e-9 * (K > 1.0 ? K : 1.0)) return -1.0;
  if (!(eps > 0.0) || group < 1 || group > 64) return -2.0;
  int n_groups = (n_cells + group - 1) / group;
  double total = 0.0;
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : total)
  for (int grp = 0; grp < n_groups; ++grp) {
    double sbar[64];
    int members = 0;
    for (int k = 0; k < group; ++k) {
      int cc = grp * group + k;
      if (cc < n_cells) ++members;
      sbar[k] = cc < n_cells ? orc_mean_strength(T[cc], n_lines, nu_line, S_ref, E_lower,
                                                 T_ref, cutoff_cm, nu0, dnu, n_nu)
                             : 0.0;
    }
    double kept = 0.0;
    for (int i = 0; i < n_lines; ++i) {
      double r = (nu_line[i] - nu0) / dnu;
      if (!orc_meets_grid(r, K, n_nu)) continue;
      double hw = orc_group_window(grp, group, n_cells, T, p, sbar, i, nu_line, S_ref,
                                   gamma_ref, n_T, E_lower, T_ref, dnu, eps, K);
      if (hw < 0.0) continue;
      double c0 = floor(r);
      double top = (double)(n_nu - 1);
      /* above: c0 + 1 .. c0 + tu; below: c0 - tl .. c0; each clipped to the grid */
      long tu = orc_last_kept(c0, +1, r, K, hw), tl = orc_last_kept(c0, -1, r, K, hw);
      if (tu >= 1) {
        double a0 = fmax(c0 + 1.0, 0.0), a1 = fmin(c0 + (double)tu, top);
        if (a1 >= a0) kept += a1 - a0 + 1.0;
      }
      if (tl >= 0) {
        double b0 = fmax(c0 - (double)tl, 0.0), b1 = fmin(c0, top);
        if (b1 >= b0) kept += b1 - b0 + 1.0;
      }
    }
    total += kept * (double)members;
  }
  return total;
}

/* ======================================================================
 * Wing return: an extension of the adaptive form (not in the paper).  The
 * points a line drops in cell c -- inside its hard window and on the grid,
 * outside the run's kept interval -- carry a Lorentz mass that the plain sum
 * would have added.  Each maximal run of consecutive dropped points a..b is
 * priced by the midpoint rule, the integral of the profile over
 * [a - 1/2, b + 1/2] in grid units:
 *   sum_{j=a..b} g / (pi ((j - r)^2 dnu^2 + g^2))
 *     ~ (atan((b + 1/2 - r) dnu / g) - atan((a - 1/2 - r) dnu / g)) / (pi dnu)
 * and the cell's total over all lines is returned as a constant over the
 * band:
 *   wing_c = u_c / (n_nu pi dnu) sum_i S_i s_ci (sum over its dropped runs
 *            of the atan differences),
 * which kappa_c(nu_j) of the adaptive form then carries at every j.
 * Returns -1 on a non-integer cutoff/dnu, -2 on bad eps or group. */
int orc_wing_return(int n_cells_listed, const int32_t* cell_list, int n_cells, const double* T,
                    const double* x, const double* p, int n_lines, const double* nu_line,
                    const double* S_ref, const double* gamma_ref, const double* n_T,
                    const double* E_lower, double T_ref, double cutoff_cm, double nu0,
                    double dnu, int n_nu, double eps, int group, double* out) {
  double Kd = cutoff_cm / dnu;
  double K = floor(Kd + 0.5);
  if (fabs(Kd - K) > 1e-9 * (K > 1.0 ? K : 1.0)) return -1;
  if (!(eps > 0.0) || group < 1 || group > 64) return -2;
#pragma omp parallel for schedule(dynamic, 1)
  for (int row = 0; row < n_cells_listed; ++row) {
    int c = cell_list[row];
    int grp = c / group;
    double sbar[64];
    for (int k = 0; k < group; ++k) {
      int cc = grp * group + k;
      sbar[k] = cc < n_cells ? orc_mean_strength(T[cc], n_lines, nu_line, S_ref, E_lower,
                                                 T_ref, cutoff_cm, nu0, dnu, n_nu)
                             : 0.0;
    }
    double total = 0.0;
    for (int i = 0; i < n_lines; ++i) {
      double r = (nu_line[i] - nu0) / dnu;
      if (!orc_meets_grid(r, K, n_nu)) continue;
      double hw = orc_group_window(grp, group, n_cells, T, p, sbar, i, nu_line, S_ref,
                                   gamma_ref, n_T, E_lower, T_ref, dnu, eps, K);
      double s = orc_strength_ratio(T[c], T_ref, nu_line[i],
                                    E_lower ? E_lower[i] : 0.0, E_lower != NULL);
      double g = orc_half_width(gamma_ref[i], n_T[i], T[c], T_ref, p[c]);
      double jlo_d = ceil(r - K) - 1.0, jhi_d = floor(r + K) + 1.0;
      long jlo = jlo_d < 0.0 ? 0 : (long)jlo_d;
      long jhi = jhi_d > (double)(n_nu - 1) ? n_nu - 1 : (long)jhi_d;
      double mass = 0.0;
      long a = -1;  /* first point of the open run of dropped points */
      for (long j = jlo; j <= jhi + 1; ++j) {
        int dropped = 0;
        if (j <= jhi) {
          double jd = (double)j;
          int hard = jd - K <= r && r <= jd + K;
          dropped = hard && !orc_kept(jd, r, K, hw);
        }
        if (dropped && a < 0) a = j;
        if (!dropped && a >= 0) {
          double b = (double)(j - 1);
          mass += atan((b + 0.5 - r) * dnu / g) - atan(((double)a - 0.5 - r) * dnu / g);
          a = -1;
        }
      }
      total += S_ref[i] * s * mass;
    }
    out[row] = orc_density(T[c], x[c], p[c]) * total / ((double)n_nu * M_PI * dnu);
  }
  return 0;
}

/* Eq. (4) in its wavenumber form: B(nu, T) = c1 nu^3 / (exp(c2 nu/T) - 1)
 * in W m^-2 sr^-1 (cm^-1)^-1, nu in cm^-1; 0 for T = 0 (cold wall). */
double orc_planck(double nu, double T) {
  if (T <= 0.0) return 0.0;
  return orc_c1() * nu * nu * nu / expm1(orc_c2() * nu / T);
}

int orc_planck_rows(int n_cells_listed, const int32_t* cell_list,
                    const double* T, double nu0, double dnu, int n_nu,
                    double* out) {
#pragma omp parallel for schedule(static)
  for (int row = 0; row < n_cells_listed; ++row) {
    double Tc = T[cell_list[row]];
    for (int j = 0; j < n_nu; ++j)
      out[(size_t)row * n_nu + j] = orc_planck(nu0 + (double)j * dnu, Tc);
  }
  return 0;
}

/* ======================================================================
 * March, Eq. (3) applied volume after volume along each ray (the paper
 * iterates one volume per step, feeding I_out back as the next I_in):
 *   I <- I e^{-tau} + B (1 - e^{-tau}),  tau = kappa l,
 * evaluated as I <- I - (I - B) a with a = -expm1(-tau), the same value in
 * exact arithmetic.  Per ray and wavenumber, with ray weight
 *   w = pi A_boundary dnu / N_rays_total   (A in m^2),
 *   entering += w I_wall;  per segment: absorbed[c] += w I a,
 *   emitted[c] += w B a;   at exit: escaped += w I.
 * balance[] accumulates (entering, emitted, absorbed, escaped); in exact
 * arithmetic entering + emitted = absorbed + escaped for every ray.
 * Loops: rays in the given order, then wavenumbers, then segments.
 * Walls are black at T_wall (0: cold).
 *
 * Rays are given explicitly (O, D) so the same routine serves Philox rays
 * and hand-placed debug rays.  kappa/planck rows are addressed through
 * cell_row (cell -> row, -1 if not supplied; NULL means row = cell).
 * exit_I, if not NULL, receives I at exit per (ray, j).
 * ==================================================================== */
int orc_march(int nx, int ny, int nz, double h_cm, int n_rays,
              const int64_t* O, const int64_t* D, double weight,
              double T_wall, double nu0, double dnu, int n_nu,
              const double* kappa, const double* planck,
              const int32_t* cell_row, double* absorbed, double* emitted,
              double balance[4], double* exit_I) {
  int cap = nx + ny + nz + 3;
  int32_t* cells = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
  double* lens = (double*)malloc(sizeof(double) * (size_t)cap);
  int32_t* rows = (int32_t*)malloc(sizeof(int32_t) * (size_t)cap);
  double* bwall = (double*)malloc(sizeof(double) * (size_t)n_nu);
  for (int j = 0; j < n_nu; ++j) bwall[j] = orc_planck(nu0 + (double)j * dnu, T_wall);
  int rc = 0;
  for (int r = 0; r < n_rays && rc == 0; ++r) {
    int ns = orc_segments(nx, ny, nz, h_cm, O + 3 * (size_t)r, D + 3 * (size_t)r,
                          cells, lens, cap);
    if (ns < 0) { rc = -1; break; }
    for (int k = 0; k < ns; ++k) {
      rows[k] = cell_row ? cell_row[cells[k]] : cells[k];
      if (rows[k] < 0) { rc = -2; break; }
    }
    if (rc) break;
    for (int j = 0; j < n_nu; ++j) {
      double I = bwall[j];
      balance[0] += weight * I;
      for (int k = 0; k < ns; ++k) {
        double kap = kappa[(size_t)rows[k] * n_nu + j];
        double B = planck[(size_t)rows[k] * n_nu + j];
        double tau = kap * lens[k];
        double a = -expm1(-tau);
        absorbed[cells[k]] += weight * I * a;
        emitted[cells[k]] += weight * B * a;
        balance[1] += weight * B * a;
        balance[2] += weight * I * a;
        I = I - (I - B) * a;
      }
      balance[3] += weight * I;
      if (exit_I) exit_I[(size_t)r * n_nu + j] = I;
    }
  }
  free(cells); free(lens); free(rows); free(bwall);
  return rc;
}

/* boundary area in m^2 of an nx x ny x nz box of cubic cells of edge h_m */
double orc_boundary_area(int nx, int ny, int nz, double h_m) {
  return 2.0 * h_m * h_m *
         ((double)nx * ny + (double)ny * nz + (double)nz * nx);
}
