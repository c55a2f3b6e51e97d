// Host construction of the moduli and CRT constants.
//
// Moduli: the hybrid list of Section III-D.  Candidates are the squares s^2
// (2 <= s <= 33) together with the integers 2..513, scanned in descending
// order; a candidate is kept when it is coprime to every kept modulus.  This
// puts 1089, 1024, 961, 841, 625, 529 first and continues 511, 509, 503, ...
// Squares use the modular-reduction split with s = sqrt(p) (Section III-C),
// the others the Karatsuba split with s = 16 (Section III-B).  The
// Karatsuba-only list of Section III-B (the same scan over 2..513 alone:
// 513, 512, 511, 509, 505, ...) uses the Karatsuba split for every modulus.
// The INT8 list of Section II (the scan over 2..256: 256, 255, 253, ...)
// keeps each residue, in [-128, 127], as one INT8 operand.
//
// Karatsuba products: the residue-product kernel sums the three digit
// products C1 = A1 B1, C2 = A2 B2, C3 = A3 B3 in one accumulator, one pass
// after the other, and folds it between passes; the combination
// 240 C1 - 15 C2 + 16 C3 (eq. C'-Karatsuba) is reached as
// c (b (a X + Y) + Z) with (X, Y, Z) the passes in order:
//   p coprime to 15: (C1, C3, C2), a = 15,  b = -16/15, c = -15
//   p odd otherwise: (C1, C2, C3), a = -16, b = -15/16, c = 16
// (the divisions modulo p).  Every modulus of the hybrid list is coprime to
// 15 (1089 = 3^2 11^2 and 625 = 5^4 precede them); of the Karatsuba-only
// list, 513 = 3^3 19 and 505 = 5 101 take the second order.
//
// CRT: with P the product of the moduli, w_l = q_l P / p_l where q_l is the
// inverse of P / p_l modulo p_l (eq. CRT_finalreduction), stored as 32-bit
// little-endian limbs.
#include <string.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "oz2_internal.h"

namespace oz2 {
namespace {

using Big = std::vector<uint32_t>;  // little-endian base-2^32 digits

int gcd_int(int a, int b) {
  while (b) {
    int t = a % b;
    a = b;
    b = t;
  }
  return a;
}

void big_mul_small(Big &x, uint32_t v) {
  uint64_t carry = 0;
  for (auto &d : x) {
    uint64_t t = (uint64_t)d * v + carry;
    d = (uint32_t)t;
    carry = t >> 32;
  }
  if (carry) x.push_back((uint32_t)carry);
}

uint32_t big_mod_small(const Big &x, uint32_t p) {
  uint64_t r = 0;
  for (size_t i = x.size(); i-- > 0;) r = ((r << 32) | x[i]) % p;
  return (uint32_t)r;
}

void big_sub_one(Big &x) {
  for (auto &d : x) {
    if (d-- != 0) break;
  }
}

void big_shr1(Big &x) {
  for (size_t i = 0; i < x.size(); ++i) {
    x[i] >>= 1;
    if (i + 1 < x.size()) x[i] |= (x[i + 1] & 1u) << 31;
  }
}

int big_bits(const Big &x) {
  for (size_t i = x.size(); i-- > 0;)
    if (x[i]) return (int)(32 * i) + 32 - __builtin_clz(x[i]);
  return 0;
}

// value of x rounded toward zero to 53 bits (round=false) or to nearest-ish
// (round=true, used only as an estimate)
double big_to_double(const Big &x, bool round) {
  int nb = big_bits(x);
  if (nb == 0) return 0.0;
  // gather the top 64 bits
  uint64_t top = 0;
  int shift = nb - 64;  // bit position of the lowest gathered bit
  for (int b = 0; b < 64; ++b) {
    int pos = shift + b;
    if (pos < 0) continue;
    uint32_t bit = (x[pos / 32] >> (pos % 32)) & 1u;
    top |= (uint64_t)bit << b;
  }
  // keep 53 bits
  int drop = 64 - 53;
  uint64_t mant = top >> drop;
  if (round && ((top >> (drop - 1)) & 1u)) mant += 1;
  return std::ldexp((double)mant, shift + drop);
}

int inv_mod(int a, int p) {  // a^{-1} mod p, gcd(a, p) = 1
  int t = 0, nt = 1, r = p, nr = a % p;
  while (nr) {
    int q = r / nr;
    int tmp = t - q * nt;
    t = nt;
    nt = tmp;
    tmp = r - q * nr;
    r = nr;
    nr = tmp;
  }
  return t < 0 ? t + p : t;
}

std::vector<int> modulus_list(int N, int list) {
  std::vector<int> cand;
  if (list == OZ2_MODULI_HYBRID)
    for (int s = 2; s <= 33; ++s) cand.push_back(s * s);
  const int top = list == OZ2_MODULI_INT8 ? 256 : 513;
  for (int v = 2; v <= top; ++v) cand.push_back(v);
  std::sort(cand.begin(), cand.end(), [](int a, int b) { return a > b; });
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  std::vector<int> out;
  for (int c : cand) {
    if ((int)out.size() == N) break;
    bool ok = true;
    for (int q : out) ok = ok && gcd_int(c, q) == 1;
    if (ok) out.push_back(c);
  }
  return out;
}

// x in the symmetric range [-floor(p/2), ceil(p/2) - 1]
int sym(int64_t x, int p) {
  int r = (int)(((x % p) + p) % p);
  return r > p - 1 - p / 2 ? r - p : r;
}

}  // namespace

bool build_tables(int N, int list, Tables *t) {
  if (N < 1 || N > kMaxN) return false;
  if (list != OZ2_MODULI_HYBRID && list != OZ2_MODULI_KARATSUBA && list != OZ2_MODULI_INT8)
    return false;
  const bool hybrid = list == OZ2_MODULI_HYBRID, int8 = list == OZ2_MODULI_INT8;
  memset(t, 0, sizeof(*t));
  std::vector<int> p = modulus_list(N, list);
  if ((int)p.size() != N) return false;
  t->N = N;
  int slice = 0;
  for (int l = 0; l < N; ++l) {
    int r = (int)std::lround(std::sqrt((double)p[l]));
    bool square = hybrid && r * r == p[l];
    // squares must form a prefix of the list (the kernels index them first)
    if (square && l != t->nsq) return false;
    if (square) t->nsq = l + 1;
    if (!square && !int8) t->nka += 1;
    t->p[l] = p[l];
    t->kind[l] = square ? 0 : (int8 ? 2 : 1);
    t->s[l] = square ? r : (int8 ? 1 : 16);
    t->slice0[l] = slice;
    slice += square ? 2 : (int8 ? 1 : 3);
    t->inv_p[l] = 1.0f / (float)p[l];
    t->inv_pd[l] = 1.0 / (double)p[l];
    t->inv_pair[l] = l + 1 < N ? 1.0 / ((double)p[l] * (double)p[l + 1]) : 0.0;
    // the residue pass's shared FP64 step needs p_l p_(l+1) < 2^21
    if (l + 1 < N && (int64_t)p[l] * p[l + 1] >= (1 << 21)) return false;
    t->inv_s[l] = 1.0f / (float)t->s[l];
    if (!square && !int8) {
      const int q = p[l];
      if (gcd_int(q, 15) == 1) {          // passes C1, C3, C2
        t->kfold[l][0] = sym(15, q);
        t->kfold[l][1] = sym((int64_t)-16 * inv_mod(15 % q, q), q);
        t->kfold[l][2] = sym(-15, q);
        t->kfold[l][3] = 2;
      } else if (q % 2 == 1) {            // passes C1, C2, C3
        t->kfold[l][0] = sym(-16, q);
        t->kfold[l][1] = sym((int64_t)-15 * inv_mod(16 % q, q), q);
        t->kfold[l][2] = sym(16, q);
        t->kfold[l][3] = 1;
      } else {
        return false;
      }
    }
    uint64_t v = 1;
    for (int e = 0; e < kPowT; ++e) {
      t->pw[l][e] = (uint16_t)v;
      v = (v * 2) % p[l];
    }
  }
  t->M = slice;

  Big P{1};
  for (int l = 0; l < N; ++l) big_mul_small(P, (uint32_t)p[l]);
  int limbs = (int)P.size();
  if (limbs + 1 > kLimbs) return false;
  t->limbs = limbs;
  for (int i = 0; i < limbs; ++i) t->P[i] = P[i];
  Big half = P;
  big_shr1(half);
  for (size_t i = 0; i < half.size(); ++i) t->half[i] = half[i];
  // top = P - 1 - half, limb by limb with borrows (P > half)
  {
    int64_t borrow = 0;
    for (int i = 0; i < limbs; ++i) {
      int64_t d = (int64_t)P[i] - (i < (int)half.size() ? (int64_t)half[i] : 0) - borrow -
                  (i == 0 ? 1 : 0);
      borrow = d < 0 ? 1 : 0;
      t->top[i] = (uint32_t)(d + (borrow << 32));
    }
    for (int i = 0; i < limbs; ++i) t->Pdl[i] = (double)P[i];
  }
  for (int l = 0; l < N; ++l) {
    Big others{1};
    for (int j = 0; j < N; ++j)
      if (j != l) big_mul_small(others, (uint32_t)p[j]);
    int q = inv_mod((int)big_mod_small(others, (uint32_t)p[l]), p[l]);
    big_mul_small(others, (uint32_t)q);
    if ((int)others.size() > limbs) return false;
    for (size_t i = 0; i < others.size(); ++i) {
      t->w[l][i] = others[i];
      t->wd[l][i] = (double)others[i];
    }
  }
  t->P_d = big_to_double(P, true);
  t->inv_P_d = 1.0 / t->P_d;
  // an estimate of C' within 2^-48 P of it (see the CRT) that is at most this
  // is below floor(P/2) - 1 in magnitude, so C' needs no range correction
  t->crt_fast = t->P_d * (0.5 - 0x1p-40) - 2.0;
  Big Pm1 = P;
  big_sub_one(Pm1);
  t->D = big_to_double(Pm1, false);
  return true;
}

}  // namespace oz2
