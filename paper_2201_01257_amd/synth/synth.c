/* Seeded, counter-based synthetic inputs for block-sparse tensor workloads.
 *
 * This module holds no arithmetic of the contraction method itself.  It produces the input
 * values (two-electron-integral-like tensors, amplitudes, orbital energies) that both the HIP
 * path and the CPU oracle consume, so that both sides see bit-identical inputs.
 *
 * Every value is a pure function of (seed, tag, linear index in the untiled dense index
 * space), so the same values exist under any tiling and any block can be generated alone.
 *
 * Random bits: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014; output function as in Vigna's public splitmix64.c), used as a
 * counter-based generator: output c of the stream with state s is mix64(s + (c+1) * gamma).
 * Uniforms take the top 53 bits.  Normals use the Box-Muller transform (Box and Muller,
 * Ann. Math. Statist. 29, 1958) on two uniforms drawn at counters 2*idx and 2*idx+1.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>

#define SYNTH_GAMMA 0x9E3779B97F4A7C15ULL
#define SYNTH_MAX_RANK 8

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static inline uint64_t splitmix_at(uint64_t state, uint64_t c) { return mix64(state + (c + 1) * SYNTH_GAMMA); }

static inline double u53(uint64_t x) { return (double)(x >> 11) * 0x1.0p-53; }

static inline double normal_at(uint64_t key, uint64_t idx) {
  double u1 = 1.0 - u53(splitmix_at(key, 2 * idx)); /* (0, 1] */
  double u2 = u53(splitmix_at(key, 2 * idx + 1));   /* [0, 1) */
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

uint64_t synth_key(uint64_t seed, uint64_t tag) { return splitmix_at(splitmix_at(seed, 0) ^ tag, 0); }

double synth_normal_at(uint64_t seed, uint64_t tag, uint64_t idx) { return normal_at(synth_key(seed, tag), idx); }

/* out[i] = a + (b - a) * U(key, first + i), i in [0, n). */
int synth_uniform(uint64_t seed, uint64_t tag, int64_t first, int64_t n, double a, double b, double* out) {
  if (n < 0 || (n > 0 && !out)) return -1;
  uint64_t key = synth_key(seed, tag);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = a + (b - a) * u53(splitmix_at(key, (uint64_t)(first + i)));
  return 0;
}

enum { SYNTH_NORMAL = 0, SYNTH_SYMMETRIC = 1, SYNTH_AMPLITUDE = 2, SYNTH_CHOLESKY = 3 };

/* Fill a dense row-major box out[ext[0]]...[ext[rank-1]] whose corner is lo[] in a tensor of
 * dense shape dims[].  nalpha[d]: indices below it have spin alpha (0), the rest beta (1).
 *
 * kind SYNTH_NORMAL:    sigma * z(idx)
 * kind SYNTH_SYMMETRIC: rank 4 only.  sigma * sum_{g in G} z(idx(g(p))) / sqrt(|G|), where G
 *                       is the subset of {id, (badc), (cdab), (dcba)} that maps the pattern of
 *                       dimension classes vclass[] onto itself (a subgroup).
 * kind SYNTH_AMPLITUDE: sigma * z(idx) / D(p) with D = sum of energy[d][p_d] over dims with
 *                       esign[d] > 0 in dimension order, then minus energy[d][p_d] over dims
 *                       with esign[d] < 0 in dimension order.
 * kind SYNTH_CHOLESKY:  rank 3 (p, q, L), p and q in one spin-orbital space of dims[0] ==
 *                       dims[1] with nalpha[0] == nalpha[1], L auxiliary.  Zero unless p and q
 *                       have the same spin; otherwise sigma * z(idx) at the index of the
 *                       unordered pair of their spatial orbitals (p - nalpha for beta) and L, so
 *                       the value is symmetric in (p, q) and equal for the alpha and beta
 *                       copies of a spatial pair (vectors of spatial-orbital integrals).
 * spin_zero != 0 sets elements that break spin conservation (first half of the dims against
 * the second half, even ranks) to exactly zero.
 */
int synth_fill(uint64_t seed, uint64_t tag, int kind, int rank, const int64_t* dims, const int64_t* nalpha,
               const int64_t* lo, const int64_t* ext, double sigma, const double* const* energy,
               const int8_t* esign, const int8_t* vclass, int spin_zero, double* out) {
  if (rank < 1 || rank > SYNTH_MAX_RANK || !dims || !lo || !ext || !out) return -1;
  if (kind == SYNTH_SYMMETRIC && (rank != 4 || !vclass)) return -1;
  if (kind == SYNTH_AMPLITUDE && (!energy || !esign)) return -1;
  if (kind == SYNTH_CHOLESKY && (rank != 3 || !nalpha || dims[0] != dims[1] || nalpha[0] != nalpha[1])) return -1;
  if (spin_zero && !nalpha) return -1;
  for (int d = 0; d < rank; ++d)
    if (lo[d] < 0 || ext[d] < 0 || lo[d] + ext[d] > dims[d]) return -1;
  int64_t rows = 1;
  for (int d = 0; d < rank - 1; ++d) rows *= ext[d];
  const int64_t inner = ext[rank - 1];
  if (rows == 0 || inner == 0) return 0;
  const uint64_t key = synth_key(seed, tag);

  static const int perms[4][4] = {{0, 1, 2, 3}, {1, 0, 3, 2}, {2, 3, 0, 1}, {3, 2, 1, 0}};
  int group[4], ngroup = 0;
  if (kind == SYNTH_SYMMETRIC) {
    for (int g = 0; g < 4; ++g) {
      int ok = 1;
      for (int d = 0; d < 4; ++d)
        if (vclass[perms[g][d]] != vclass[d] || dims[perms[g][d]] != dims[d]) ok = 0;
      if (ok) group[ngroup++] = g;
    }
  }
  const double gscale = ngroup > 0 ? 1.0 / sqrt((double)ngroup) : 1.0;

#pragma omp parallel for schedule(static)
  for (int64_t row = 0; row < rows; ++row) {
    int64_t p[SYNTH_MAX_RANK];
    int64_t rem = row;
    for (int d = rank - 2; d >= 0; --d) {
      p[d] = lo[d] + rem % ext[d];
      rem /= ext[d];
    }
    double* o = out + row * inner;
    for (int64_t c = 0; c < inner; ++c) {
      p[rank - 1] = lo[rank - 1] + c;
      if (spin_zero && (rank % 2) == 0) {
        int s0 = 0, s1 = 0;
        for (int d = 0; d < rank / 2; ++d) s0 += p[d] >= nalpha[d];
        for (int d = rank / 2; d < rank; ++d) s1 += p[d] >= nalpha[d];
        if (s0 != s1) {
          o[c] = 0.0;
          continue;
        }
      }
      double v;
      if (kind == SYNTH_CHOLESKY) {
        const int64_t na = nalpha[0], nsp = na > dims[0] - na ? na : dims[0] - na;
        const int b0 = p[0] >= na, b1 = p[1] >= na;
        if (b0 != b1) {
          o[c] = 0.0;
          continue;
        }
        const int64_t s0 = p[0] - (b0 ? na : 0), s1 = p[1] - (b1 ? na : 0);
        const int64_t lo_s = s0 < s1 ? s0 : s1, hi_s = s0 < s1 ? s1 : s0;
        const uint64_t lin = ((uint64_t)lo_s * (uint64_t)nsp + (uint64_t)hi_s) * (uint64_t)dims[2] + (uint64_t)p[2];
        v = sigma * normal_at(key, lin);
      } else if (kind == SYNTH_SYMMETRIC) {
        /* orbit members summed in ascending linear index, so every member of an orbit gets the
         * bitwise-identical value */
        uint64_t lins[4];
        for (int gi = 0; gi < ngroup; ++gi) {
          const int* pg = perms[group[gi]];
          uint64_t lin = 0;
          for (int d = 0; d < 4; ++d) lin = lin * (uint64_t)dims[d] + (uint64_t)p[pg[d]];
          int pos = gi;
          while (pos > 0 && lins[pos - 1] > lin) {
            lins[pos] = lins[pos - 1];
            --pos;
          }
          lins[pos] = lin;
        }
        double s = 0.0;
        for (int gi = 0; gi < ngroup; ++gi) s += normal_at(key, lins[gi]);
        v = sigma * s * gscale;
      } else {
        uint64_t lin = 0;
        for (int d = 0; d < rank; ++d) lin = lin * (uint64_t)dims[d] + (uint64_t)p[d];
        v = sigma * normal_at(key, lin);
        if (kind == SYNTH_AMPLITUDE) {
          double den = 0.0;
          int first = 1;
          for (int d = 0; d < rank; ++d)
            if (esign[d] > 0) {
              den = first ? energy[d][p[d]] : den + energy[d][p[d]];
              first = 0;
            }
          for (int d = 0; d < rank; ++d)
            if (esign[d] < 0) den = first ? -energy[d][p[d]] : den - energy[d][p[d]], first = 0;
          v = v / den;
        }
      }
      o[c] = v;
    }
  }
  return 0;
}
