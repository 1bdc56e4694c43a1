// CPU oracle for extended-stabilizer generator propagation -- TEST INFRASTRUCTURE.
//
// Only the tests, the smoke check and the benchmark's CPU-baseline leg may load this
// library. The product path never calls it, and it shares no code with the HIP path:
// its gate tables, Pauli algebra, merge and ordering are written here independently.
//
// What it computes (paper: Sec. II-A, eq. (1) and the sentence after it; Sec. II-C):
//   the n stabilizer generators of |0^n> start as Z_j = I..I Z I..I (qubit j holds Z),
//   and every gate g of the circuit, taken in instruction order, replaces each
//   generator G by g G g^dagger. A generator is a real linear combination of Pauli
//   strings, held here as a list of (x bits, z bits, weight) terms.
//
// Algorithm: the paper's "v1" propagation (Sec. I, Sec. V), gate by gate:
//   * a one-qubit gate on wire q maps the local Pauli p of every term to
//     sum_a R[a][p] sigma_a, where R is the gate's real Pauli transfer matrix
//     R[a][b] = (1/2) Tr(sigma_a U sigma_b U^dagger); identity stays identity;
//   * CX and CZ act on the two local Paulis as signed permutations (Sec. III-C-2);
//   * a two-qubit rotation exp(-i t A / 2), A = P (x) P for P in {X, Y, Z}, keeps a Pauli
//     string Q that commutes with A and sends one that anticommutes to
//     cos t Q + sin t (-i A Q) (-i A Q is again a Pauli string, with a real sign);
//     ISWAP = exp(i pi/4 (XX + YY)) is the two rotations at t = -pi/2 (cos exactly 0),
//     a signed permutation;
//   * after a gate that is not a signed permutation, images with equal Pauli
//     strings are summed ("index-based Pauli accumulation", abstract) and exact
//     zeros are dropped (only non-zero weights are stored, Sec. III-B);
//   * at the end of each circuit layer, terms with |w| <= eps are dropped.
// Generators never interact, so they are processed independently (OpenMP over
// generators); that changes no result.
//
// Conventions: Pauli codes I=0, X=1, Y=2, Z=3 (Sec. III-B); bit q of x / z is
// qubit q; X=(x1,z0), Y=(x1,z1), Z=(x0,z1). Rotations R_s(t) = exp(-i t s / 2).
// Output order: ascending by the paper's base-4 index sum_j d_j 4^(n-1-j), qubit 0
// the most significant digit (Sec. III-B, Example 1).
//
// Every function below is pinned by tests against values the paper prints (CX rules,
// worked examples), dense statevector / unitary brute force, a stabilizer tableau, and
// closed-form term counts; nothing here is "parity unpinned".

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

struct Term {
  uint64_t x, z;
  double w;
};

// Gate codes of the instruction arrays (the input format).
enum GateCode {
  G_H = 0, G_S = 1, G_SDG = 2, G_T = 3, G_TDG = 4, G_SX = 5, G_X = 6, G_Y = 7, G_Z = 8,
  G_RX = 9, G_RY = 10, G_RZ = 11, G_CX = 12, G_CZ = 13, G_ISWAP = 14, G_RXX = 15, G_RYY = 16,
  G_RZZ = 17, G_COUNT = 18
};

inline bool two_qubit(int code) { return code >= G_CX && code <= G_RZZ; }

inline int local_pauli(const Term& t, int q) {
  int xb = (int)((t.x >> q) & 1u), zb = (int)((t.z >> q) & 1u);
  if (!xb && !zb) return 0;
  if (xb && !zb) return 1;
  if (xb && zb) return 2;
  return 3;
}

inline void set_local_pauli(Term& t, int q, int p) {
  uint64_t m = 1ull << q;
  t.x &= ~m;
  t.z &= ~m;
  if (p == 1 || p == 2) t.x |= m;
  if (p == 2 || p == 3) t.z |= m;
}

// Real Pauli transfer matrix of a one-qubit gate, R[out][in] over (I, X, Y, Z).
// Each entry is the closed form of (1/2) Tr(sigma_out U sigma_in U^dagger) for the
// gate's unitary; the rotation blocks are the SO(3) rotations by t about the axis.
bool ptm_1q(int code, double theta, double R[4][4]) {
  std::memset(R, 0, sizeof(double) * 16);
  R[0][0] = 1.0;
  auto rot = [&](int axis, double t) {
    // rotation of the (X, Y, Z) Bloch components by angle t about `axis` (1=X,2=Y,3=Z)
    double c = std::cos(t), s = std::sin(t);
    int a = axis, b = axis % 3 + 1, d = b % 3 + 1;  // cyclic (a, b, d)
    R[a][a] = 1.0;
    R[b][b] = c;
    R[d][d] = c;
    R[d][b] = s;   // sigma_b -> c sigma_b + s sigma_d
    R[b][d] = -s;  // sigma_d -> c sigma_d - s sigma_b
  };
  switch (code) {
    case G_H: R[3][1] = 1; R[2][2] = -1; R[1][3] = 1; return true;   // X<->Z, Y->-Y
    case G_S: R[2][1] = 1; R[1][2] = -1; R[3][3] = 1; return true;   // X->Y, Y->-X
    case G_SDG: R[2][1] = -1; R[1][2] = 1; R[3][3] = 1; return true; // X->-Y, Y->X
    case G_SX: R[1][1] = 1; R[3][2] = 1; R[2][3] = -1; return true;  // Y->Z, Z->-Y
    case G_X: R[1][1] = 1; R[2][2] = -1; R[3][3] = -1; return true;
    case G_Y: R[1][1] = -1; R[2][2] = 1; R[3][3] = -1; return true;
    case G_Z: R[1][1] = -1; R[2][2] = -1; R[3][3] = 1; return true;
    case G_T: rot(3, M_PI / 4.0); return true;
    case G_TDG: rot(3, -M_PI / 4.0); return true;
    case G_RX: rot(1, theta); return true;
    case G_RY: rot(2, theta); return true;
    case G_RZ: rot(3, theta); return true;
    default: return false;
  }
}

// Two-qubit Clifford gates as updates of the symplectic bits with a sign
// (Aaronson & Gottesman 2004). Returns true when the sign flips.
inline bool apply_cx(Term& t, int c, int tg) {
  uint64_t xc = (t.x >> c) & 1u, zc = (t.z >> c) & 1u;
  uint64_t xt = (t.x >> tg) & 1u, zt = (t.z >> tg) & 1u;
  bool flip = (xc & zt & (xt ^ zc ^ 1u)) != 0;
  xt ^= xc;
  zc ^= zt;
  t.x = (t.x & ~(1ull << tg)) | (xt << tg);
  t.z = (t.z & ~(1ull << c)) | (zc << c);
  return flip;
}

inline bool apply_cz(Term& t, int a, int b) {
  uint64_t xa = (t.x >> a) & 1u, za = (t.z >> a) & 1u;
  uint64_t xb = (t.x >> b) & 1u, zb = (t.z >> b) & 1u;
  bool flip = (xa & xb & (za ^ zb)) != 0;
  za ^= xb;
  zb ^= xa;
  t.z = (t.z & ~(1ull << a)) | (za << a);
  t.z = (t.z & ~(1ull << b)) | (zb << b);
  return flip;
}

bool is_signed_permutation(const double* R, int dim) {
  for (int col = 0; col < dim; ++col) {
    int nz = 0;
    for (int row = 0; row < dim; ++row) {
      double v = R[row * dim + col];
      if (v != 0.0) {
        if (v != 1.0 && v != -1.0) return false;
        ++nz;
      }
    }
    if (nz != 1) return false;
  }
  return true;
}

bool key_less(const Term& a, const Term& b) {
  if (a.x != b.x) return a.x < b.x;
  return a.z < b.z;
}

// Sum the weights of images that carry the same Pauli string; keep non-zero sums.
void merge_into(std::vector<Term>& images, std::vector<Term>& out) {
  std::stable_sort(images.begin(), images.end(), key_less);
  out.clear();
  size_t i = 0;
  while (i < images.size()) {
    Term acc = images[i];
    size_t j = i + 1;
    while (j < images.size() && images[j].x == acc.x && images[j].z == acc.z) {
      acc.w += images[j].w;
      ++j;
    }
    if (acc.w != 0.0) out.push_back(acc);
    i = j;
  }
}

// Phase exponent e of a product of two one-qubit Paulis given by their (x, z) bits:
// P1 P2 = i^e P3 with P3 = (x1 ^ x2, z1 ^ z2) (Aaronson & Gottesman 2004, function g).
inline int product_phase(int x1, int z1, int x2, int z2) {
  if (!x1 && !z1) return 0;
  if (x1 && z1) return z2 - x2;
  if (x1) return z2 * (2 * x2 - 1);
  return x2 * (1 - 2 * z2);
}

// exp(-i t A / 2), A = P (x) P on wires (a, b), P given by its bits (px, pz); c = cos t and
// s = sin t are passed in (exact 0 / -1 for ISWAP). A term that anticommutes with A gains
// the image s * (-i A Q); with c == 0 it is replaced by it.
void apply_pp_rotation(std::vector<Term>& gen, int a, int b, int px, int pz, double c, double s,
                       std::vector<Term>& scratch) {
  scratch.clear();
  for (const Term& t : gen) {
    const int xa = (int)((t.x >> a) & 1u), za = (int)((t.z >> a) & 1u);
    const int xb = (int)((t.x >> b) & 1u), zb = (int)((t.z >> b) & 1u);
    // symplectic product of Q with A: odd = anticommute
    const int sym = ((xa & pz) ^ (za & px)) ^ ((xb & pz) ^ (zb & px));
    if (!sym) {
      scratch.push_back(t);
      continue;
    }
    if (c != 0.0) scratch.push_back(Term{t.x, t.z, t.w * c});
    // -i A Q = i^(e - 1) (A Q) with e the phase exponent of A Q; e is odd here
    const int e = product_phase(px, pz, xa, za) + product_phase(px, pz, xb, zb);
    const int k = ((e - 1) % 4 + 4) % 4;  // 0 or 2
    Term u = t;
    u.x ^= ((uint64_t)px << a) | ((uint64_t)px << b);
    u.z ^= ((uint64_t)pz << a) | ((uint64_t)pz << b);
    u.w = t.w * s * (k == 0 ? 1.0 : -1.0);
    scratch.push_back(u);
  }
  if (c == 0.0) {
    gen.swap(scratch);  // a signed permutation: no two images share a string
  } else {
    std::vector<Term> out;
    merge_into(scratch, out);
    gen.swap(out);
  }
}

void apply_2q_gate(std::vector<Term>& gen, int code, int a, int b, double theta, std::vector<Term>& scratch) {
  switch (code) {
    case G_ISWAP:
      apply_pp_rotation(gen, a, b, 1, 0, 0.0, -1.0, scratch);  // exp(i pi/4 XX)
      apply_pp_rotation(gen, a, b, 1, 1, 0.0, -1.0, scratch);  // exp(i pi/4 YY)
      return;
    case G_RXX: apply_pp_rotation(gen, a, b, 1, 0, std::cos(theta), std::sin(theta), scratch); return;
    case G_RYY: apply_pp_rotation(gen, a, b, 1, 1, std::cos(theta), std::sin(theta), scratch); return;
    case G_RZZ: apply_pp_rotation(gen, a, b, 0, 1, std::cos(theta), std::sin(theta), scratch); return;
    default: return;
  }
}

// Generic one-qubit map given by a 4x4 matrix R[out][in].
void apply_map_1q(std::vector<Term>& gen, int q, const double R[4][4], std::vector<Term>& scratch) {
  double flat[16];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) flat[a * 4 + b] = R[a][b];
  if (is_signed_permutation(flat, 4)) {
    for (Term& t : gen) {
      int p = local_pauli(t, q);
      for (int a = 0; a < 4; ++a) {
        if (R[a][p] != 0.0) {
          set_local_pauli(t, q, a);
          t.w *= R[a][p];
          break;
        }
      }
    }
    return;
  }
  scratch.clear();
  for (const Term& t : gen) {
    int p = local_pauli(t, q);
    for (int a = 0; a < 4; ++a) {
      double r = R[a][p];
      if (r == 0.0) continue;
      Term u = t;
      set_local_pauli(u, q, a);
      u.w = t.w * r;
      scratch.push_back(u);
    }
  }
  merge_into(scratch, gen);
}

// Generic two-qubit map given by a 16x16 matrix R[out][in]; local index 4*p(q0) + p(q1).
void apply_map_2q(std::vector<Term>& gen, int q0, int q1, const double* R, std::vector<Term>& scratch) {
  bool perm = is_signed_permutation(R, 16);
  scratch.clear();
  for (const Term& t : gen) {
    int in = 4 * local_pauli(t, q0) + local_pauli(t, q1);
    for (int a = 0; a < 16; ++a) {
      double r = R[a * 16 + in];
      if (r == 0.0) continue;
      Term u = t;
      set_local_pauli(u, q0, a >> 2);
      set_local_pauli(u, q1, a & 3);
      u.w = t.w * r;
      scratch.push_back(u);
    }
  }
  if (perm) {
    gen.swap(scratch);
  } else {
    merge_into(scratch, gen);
  }
}

void apply_gate(std::vector<Term>& gen, int code, int q0, int q1, double theta,
                std::vector<Term>& scratch) {
  if (code == G_CX) {
    for (Term& t : gen)
      if (apply_cx(t, q0, q1)) t.w = -t.w;
    return;
  }
  if (code == G_CZ) {
    for (Term& t : gen)
      if (apply_cz(t, q0, q1)) t.w = -t.w;
    return;
  }
  if (two_qubit(code)) {
    apply_2q_gate(gen, code, q0, q1, theta, scratch);
    return;
  }
  double R[4][4];
  ptm_1q(code, theta, R);
  apply_map_1q(gen, q0, R, scratch);
}

void prune(std::vector<Term>& gen, double eps) {
  size_t k = 0;
  for (size_t i = 0; i < gen.size(); ++i)
    if (std::fabs(gen[i].w) > eps) gen[k++] = gen[i];
  gen.resize(k);
}

// Paper index order: compare digit by digit from qubit 0 (most significant).
bool paper_order_less(const Term& a, const Term& b, int n) {
  for (int q = 0; q < n; ++q) {
    int pa = local_pauli(a, q), pb = local_pauli(b, q);
    if (pa != pb) return pa < pb;
  }
  return false;
}

}  // namespace

struct oracle_state {
  int n;
  std::vector<int> gen_ids;                 // which generator Z_j each slot started from
  std::vector<std::vector<Term>> gens;
};

extern "C" {

oracle_state* oracle_new_subset(int n, int k, const int* gens) {
  if (n < 1 || n > 64 || k < 0) return nullptr;
  oracle_state* s = new oracle_state;
  s->n = n;
  for (int i = 0; i < k; ++i) {
    int j = gens[i];
    if (j < 0 || j >= n) {
      delete s;
      return nullptr;
    }
    s->gen_ids.push_back(j);
    std::vector<Term> g(1);
    g[0].x = 0;
    g[0].z = 1ull << j;  // Z on qubit j
    g[0].w = 1.0;
    s->gens.push_back(std::move(g));
  }
  return s;
}

oracle_state* oracle_new(int n) {
  if (n < 1 || n > 64) return nullptr;
  std::vector<int> all(n);
  for (int j = 0; j < n; ++j) all[j] = j;
  return oracle_new_subset(n, n, all.data());
}

// Arbitrary starting generators (used to replay the paper's Example 1).
oracle_state* oracle_new_terms(int n, int n_gens, const uint64_t* gen_off, const uint64_t* x,
                               const uint64_t* z, const double* w) {
  if (n < 1 || n > 64 || n_gens < 0) return nullptr;
  oracle_state* s = new oracle_state;
  s->n = n;
  for (int g = 0; g < n_gens; ++g) {
    s->gen_ids.push_back(g);
    std::vector<Term> v;
    for (uint64_t i = gen_off[g]; i < gen_off[g + 1]; ++i) v.push_back(Term{x[i], z[i], w[i]});
    s->gens.push_back(std::move(v));
  }
  return s;
}

void oracle_free(oracle_state* s) { delete s; }

int oracle_num_gens(const oracle_state* s) { return (int)s->gens.size(); }

static bool valid_gate(const oracle_state* s, int code, int q0, int q1) {
  if (code < 0 || code >= G_COUNT) return false;
  if (q0 < 0 || q0 >= s->n) return false;
  if (two_qubit(code)) {
    if (q1 < 0 || q1 >= s->n || q1 == q0) return false;
  }
  return true;
}

int oracle_gate(oracle_state* s, int code, int q0, int q1, double theta) {
  if (!valid_gate(s, code, q0, q1)) return -1;
  std::vector<Term> scratch;
  for (auto& g : s->gens) apply_gate(g, code, q0, q1, theta, scratch);
  return 0;
}

int oracle_ptm1(oracle_state* s, int q, const double* R16) {
  if (q < 0 || q >= s->n) return -1;
  double R[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) R[a][b] = R16[a * 4 + b];
  std::vector<Term> scratch;
  for (auto& g : s->gens) apply_map_1q(g, q, R, scratch);
  return 0;
}

int oracle_ptm2(oracle_state* s, int q0, int q1, const double* R256) {
  if (q0 < 0 || q0 >= s->n || q1 < 0 || q1 >= s->n || q0 == q1) return -1;
  std::vector<Term> scratch;
  for (auto& g : s->gens) apply_map_2q(g, q0, q1, R256, scratch);
  return 0;
}

void oracle_prune(oracle_state* s, double eps) {
  for (auto& g : s->gens) prune(g, eps);
}

// Whole circuit, gate by gate, each generator on its own thread.
int oracle_run(oracle_state* s, size_t m, const uint8_t* gate, const uint32_t* q0,
               const uint32_t* q1, const double* theta, size_t n_layers, const int64_t* layer_end,
               double eps, int threads) {
  for (size_t i = 0; i < m; ++i)
    if (!valid_gate(s, gate[i], (int)q0[i], (int)q1[i])) return -1;
  for (size_t l = 0; l < n_layers; ++l)
    if (layer_end[l] < 0 || (size_t)layer_end[l] > m || (l && layer_end[l] < layer_end[l - 1])) return -1;
  const int G = (int)s->gens.size();
#ifdef _OPENMP
  if (threads < 1) threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
#endif
  for (int gi = 0; gi < G; ++gi) {
    std::vector<Term>& gen = s->gens[gi];
    std::vector<Term> scratch;
    size_t start = 0;
    for (size_t l = 0; l < n_layers; ++l) {
      size_t stop = (size_t)layer_end[l];
      for (size_t i = start; i < stop; ++i) apply_gate(gen, gate[i], (int)q0[i], (int)q1[i], theta[i], scratch);
      prune(gen, eps);
      start = stop;
    }
  }
  (void)threads;
  return 0;
}

// Gates gate[0..m) applied to every generator in order (no prune), generators in parallel.
int oracle_gates(oracle_state* s, size_t m, const uint8_t* gate, const uint32_t* q0, const uint32_t* q1,
                 const double* theta, int threads) {
  for (size_t i = 0; i < m; ++i)
    if (!valid_gate(s, gate[i], (int)q0[i], (int)q1[i])) return -1;
  const int G = (int)s->gens.size();
#ifdef _OPENMP
  if (threads < 1) threads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 1) num_threads(threads)
#endif
  for (int gi = 0; gi < G; ++gi) {
    std::vector<Term> scratch;
    for (size_t i = 0; i < m; ++i) apply_gate(s->gens[gi], gate[i], (int)q0[i], (int)q1[i], theta[i], scratch);
  }
  (void)threads;
  return 0;
}

// The number of images an operator acting on wires[0..k) produces from each generator's
// current terms: sum over terms of prod_i nnz[4*i + p_i], p_i the term's Pauli on wires[i]
// and nnz[4*i + p] the number of nonzero entries in column p of that wire's transfer
// matrix (the count a term update is defined by). out[g] per generator slot.
void oracle_fanout_sum(const oracle_state* s, int k, const int* wires, const uint8_t* nnz, uint64_t* out) {
  for (size_t g = 0; g < s->gens.size(); ++g) {
    uint64_t tot = 0;
    for (const Term& t : s->gens[g]) {
      uint64_t f = 1;
      for (int i = 0; i < k; ++i) f *= nnz[4 * i + local_pauli(t, wires[i])];
      tot += f;
    }
    out[g] = tot;
  }
}

// As oracle_fanout_sum for one two-qubit operator on wires (a, b): nnz16[4*p(a) + p(b)] is
// the number of nonzero entries of that column of its transfer matrix.
void oracle_fanout_sum2(const oracle_state* s, int a, int b, const uint8_t* nnz16, uint64_t* out) {
  for (size_t g = 0; g < s->gens.size(); ++g) {
    uint64_t tot = 0;
    for (const Term& t : s->gens[g]) tot += nnz16[4 * local_pauli(t, a) + local_pauli(t, b)];
    out[g] = tot;
  }
}

size_t oracle_count(const oracle_state* s, int g) {
  if (g < 0 || g >= (int)s->gens.size()) return 0;
  return s->gens[g].size();
}

int oracle_gen_id(const oracle_state* s, int g) {
  if (g < 0 || g >= (int)s->gens.size()) return -1;
  return s->gen_ids[g];
}

// Copy generator g out, ascending by the paper's base-4 index.
void oracle_read(const oracle_state* s, int g, uint64_t* x, uint64_t* z, double* w) {
  if (g < 0 || g >= (int)s->gens.size()) return;
  std::vector<Term> v = s->gens[g];
  const int n = s->n;
  std::sort(v.begin(), v.end(), [n](const Term& a, const Term& b) { return paper_order_less(a, b, n); });
  for (size_t i = 0; i < v.size(); ++i) {
    x[i] = v[i].x;
    z[i] = v[i].z;
    w[i] = v[i].w;
  }
}

// The transfer matrix the oracle uses for a gate: 4x4 (one-qubit) or 16x16 (two-qubit)
// R[out][in]; the two-qubit index is 4*p(q0) + p(q1). Returns the dimension, or 0.
int oracle_gate_ptm(int code, double theta, double* R) {
  if (two_qubit(code) && code != G_CX && code != G_CZ) {
    std::memset(R, 0, sizeof(double) * 256);
    std::vector<Term> gen, scratch;
    for (int in = 0; in < 16; ++in) {
      Term t{0, 0, 1.0};
      set_local_pauli(t, 0, in >> 2);
      set_local_pauli(t, 1, in & 3);
      gen.assign(1, t);
      apply_2q_gate(gen, code, 0, 1, theta, scratch);
      for (const Term& u : gen) R[(4 * local_pauli(u, 0) + local_pauli(u, 1)) * 16 + in] += u.w;
    }
    return 16;
  }
  if (code == G_CX || code == G_CZ) {
    std::memset(R, 0, sizeof(double) * 256);
    for (int in = 0; in < 16; ++in) {
      Term t{0, 0, 1.0};
      set_local_pauli(t, 0, in >> 2);
      set_local_pauli(t, 1, in & 3);
      bool flip = (code == G_CX) ? apply_cx(t, 0, 1) : apply_cz(t, 0, 1);
      int out = 4 * local_pauli(t, 0) + local_pauli(t, 1);
      R[out * 16 + in] = flip ? -1.0 : 1.0;
    }
    return 16;
  }
  double M[4][4];
  if (!ptm_1q(code, theta, M)) return 0;
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) R[a * 4 + b] = M[a][b];
  return 4;
}

}  // extern "C"
