// lz_learn.cpp -- host side of the learned per-block threshold selector.
//
// The paper finds 12/16/24/32 a good setting on its data, with the best
// tuple data-dependent at the margin (Sec. 4.3, Sec. 6).  A small network
// (64 -> 128 -> 128 -> 16, ReLU, softmax) picks one of 16 candidate tuples
// per LZ block from the block's match-length / distance-class histogram,
// trained on labels the method produces itself: every training block encoded
// under every tuple (entropy-bound sizes) and decoded on the GPU (times).
// This file holds the selector object and its file format, the labels (a
// least-squares decode-time model and the cost J), the validation table of
// the fallback rule, inference, and the learned mode of the encoder.  The
// network is trained by the GPU kernels of lz_mlp.hip.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "lz_internal.h"

using namespace lz;

namespace {

constexpr char kSelMagic[8] = {'L', 'Z', 'S', 'E', 'L', '0', '0', '1'};
constexpr uint64_t W1 = 0, B1 = W1 + kSelIn * kSelHidden, W2 = B1 + kSelHidden, B2 = W2 + kSelHidden * kSelHidden,
                   W3 = B2 + kSelHidden, B3 = W3 + kSelHidden * kSelTuples;

// SplitMix64 (Steele, Lea, Flood), the seed generator of this file.
uint64_t splitmix64(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// A standard normal deviate by the Box-Muller transform.
double normal01(uint64_t& s) {
  const double u1 = ((splitmix64(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = (splitmix64(s) >> 11) * (1.0 / 9007199254740992.0);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// Softmax probabilities of one row's 16 logits (double).
void forward_row(const lz_selector* s, const float* f, double* prob) {
  const float* P = s->params.data();
  double x[kSelIn], h1[kSelHidden], h2[kSelHidden], z[kSelTuples];
  for (uint32_t i = 0; i < kSelIn; ++i) x[i] = (double(f[i]) - s->mu[i]) / s->sd[i];
  for (uint32_t j = 0; j < kSelHidden; ++j) {
    double a = P[B1 + j];
    for (uint32_t i = 0; i < kSelIn; ++i) a += x[i] * P[W1 + i * kSelHidden + j];
    h1[j] = a > 0 ? a : 0;
  }
  for (uint32_t j = 0; j < kSelHidden; ++j) {
    double a = P[B2 + j];
    for (uint32_t i = 0; i < kSelHidden; ++i) a += h1[i] * P[W2 + i * kSelHidden + j];
    h2[j] = a > 0 ? a : 0;
  }
  double mx = -1e300;
  for (uint32_t j = 0; j < kSelTuples; ++j) {
    double a = P[B3 + j];
    for (uint32_t i = 0; i < kSelHidden; ++i) a += h2[i] * P[W3 + i * kSelTuples + j];
    z[j] = a;
    mx = std::max(mx, a);
  }
  double sum = 0;
  for (uint32_t j = 0; j < kSelTuples; ++j) sum += (prob[j] = exp(z[j] - mx));
  for (uint32_t j = 0; j < kSelTuples; ++j) prob[j] /= sum;
}

uint32_t argmax16(const double* p) {
  uint32_t k = 0;
  for (uint32_t j = 1; j < kSelTuples; ++j)
    if (p[j] > p[k]) k = j;
  return k;
}

// Solves the symmetric positive semi-definite system A c = b (n <= 8) by
// Gaussian elimination with partial pivoting; a pivot below tol leaves its
// unknown at 0 (least squares with dependent columns).
void solve_small(int n, double* A, double* b, double* c) {
  bool used[8] = {false};
  for (int col = 0; col < n; ++col) {
    int best = -1;
    double bv = 0;
    for (int r = col; r < n; ++r)
      if (fabs(A[r * n + col]) > bv) bv = fabs(A[r * n + col]), best = r;
    if (best < 0 || bv < 1e-12 * (1.0 + fabs(A[col * n + col]))) continue;
    if (best != col) {
      for (int k = 0; k < n; ++k) std::swap(A[best * n + k], A[col * n + k]);
      std::swap(b[best], b[col]);
    }
    used[col] = true;
    for (int r = 0; r < n; ++r) {
      if (r == col) continue;
      const double f = A[r * n + col] / A[col * n + col];
      if (f == 0) continue;
      for (int k = 0; k < n; ++k) A[r * n + k] -= f * A[col * n + k];
      b[r] -= f * b[col];
    }
  }
  for (int i = 0; i < n; ++i) c[i] = used[i] ? b[i] / A[i * n + i] : 0.0;
}

}  // namespace

extern "C" {

int lz_selector_create(const uint32_t* tuples, uint32_t fixed, uint64_t seed, lz_selector** out) {
  if (!tuples || !out) return fail(LZ_E_INVAL, "null argument");
  if (fixed >= kSelTuples) return fail(LZ_E_INVAL, "fixed tuple index %u >= %u", fixed, kSelTuples);
  for (uint32_t t = 0; t < kSelTuples; ++t)
    for (int k = 0; k < 4; ++k)
      if (tuples[4 * t + k] < 1) return fail(LZ_E_INVAL, "thresholds must be >= 1");
  lz_selector* s = new lz_selector();
  memcpy(s->tuples, tuples, sizeof(s->tuples));
  s->fixed = fixed;
  for (uint32_t i = 0; i < kSelIn; ++i) s->mu[i] = 0.f, s->sd[i] = 1.f;
  for (uint32_t t = 0; t < kSelTuples; ++t) s->val_J[t] = 1.f;
  // He initialisation of the weights (std sqrt(2 / fan_in)), zero biases
  s->params.assign(kSelParams, 0.f);
  uint64_t st = seed;
  const struct {
    uint64_t off, count, fan_in;
  } layers[3] = {{W1, kSelIn * kSelHidden, kSelIn}, {W2, kSelHidden * kSelHidden, kSelHidden},
                 {W3, kSelHidden * kSelTuples, kSelHidden}};
  for (const auto& L : layers)
    for (uint64_t i = 0; i < L.count; ++i) s->params[L.off + i] = float(normal01(st) * sqrt(2.0 / L.fan_in));
  *out = s;
  return 0;
}

void lz_selector_free(lz_selector* s) { delete s; }

int lz_selector_params(lz_selector* s, float* get, const float* set) {
  if (!s) return fail(LZ_E_INVAL, "null selector");
  if (get) memcpy(get, s->params.data(), 4 * kSelParams);
  if (set) memcpy(s->params.data(), set, 4 * kSelParams);
  return 0;
}

int lz_selector_info(const lz_selector* s, uint32_t* tuples, uint32_t* fixed, float* mu, float* sd, float* val_J) {
  if (!s) return fail(LZ_E_INVAL, "null selector");
  if (tuples) memcpy(tuples, s->tuples, sizeof(s->tuples));
  if (fixed) *fixed = s->fixed;
  if (mu) memcpy(mu, s->mu, sizeof(s->mu));
  if (sd) memcpy(sd, s->sd, sizeof(s->sd));
  if (val_J) memcpy(val_J, s->val_J, sizeof(s->val_J));
  return 0;
}

int lz_selector_save(const lz_selector* s, const char* path) {
  if (!s || !path) return fail(LZ_E_INVAL, "null argument");
  FILE* f = fopen(path, "wb");
  if (!f) return fail(LZ_E_INVAL, "cannot open %s for writing", path);
  const uint32_t nt = kSelTuples, np = (uint32_t)kSelParams;
  bool ok = fwrite(kSelMagic, 1, 8, f) == 8 && fwrite(&nt, 4, 1, f) == 1 && fwrite(&s->fixed, 4, 1, f) == 1 &&
            fwrite(s->tuples, sizeof(s->tuples), 1, f) == 1 && fwrite(s->mu, sizeof(s->mu), 1, f) == 1 &&
            fwrite(s->sd, sizeof(s->sd), 1, f) == 1 && fwrite(s->val_J, sizeof(s->val_J), 1, f) == 1 &&
            fwrite(&np, 4, 1, f) == 1 && fwrite(s->params.data(), 4, kSelParams, f) == kSelParams;
  ok = (fclose(f) == 0) && ok;
  return ok ? 0 : fail(LZ_E_INVAL, "writing %s failed", path);
}

int lz_selector_load(const char* path, lz_selector** out) {
  if (!path || !out) return fail(LZ_E_INVAL, "null argument");
  *out = nullptr;
  FILE* f = fopen(path, "rb");
  if (!f) return fail(LZ_E_INVAL, "cannot open %s", path);
  lz_selector* s = new lz_selector();
  char magic[8];
  uint32_t nt = 0, np = 0;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kSelMagic, 8) == 0 && fread(&nt, 4, 1, f) == 1 &&
            nt == kSelTuples && fread(&s->fixed, 4, 1, f) == 1 && s->fixed < kSelTuples &&
            fread(s->tuples, sizeof(s->tuples), 1, f) == 1 && fread(s->mu, sizeof(s->mu), 1, f) == 1 &&
            fread(s->sd, sizeof(s->sd), 1, f) == 1 && fread(s->val_J, sizeof(s->val_J), 1, f) == 1 &&
            fread(&np, 4, 1, f) == 1 && np == kSelParams;
  if (ok) {
    s->params.resize(kSelParams);
    ok = fread(s->params.data(), 4, kSelParams, f) == kSelParams;
  }
  fclose(f);
  for (uint32_t t = 0; ok && t < kSelTuples; ++t)
    for (int k = 0; k < 4; ++k) ok = ok && s->tuples[t][k] >= 1;
  for (uint32_t i = 0; ok && i < kSelIn; ++i) ok = s->sd[i] > 0.f;
  if (!ok) {
    delete s;
    return fail(LZ_E_CORRUPT, "%s is not a selector file", path);
  }
  *out = s;
  return 0;
}

int lz_learn_labels(uint32_t n_files, const uint32_t* file_blocks, uint32_t fixed, const double* size,
                    const uint64_t* counts, const double* file_ms, const uint32_t* file_depths, double lambda,
                    double* coef, double* J, int32_t* labels) {
  if (!n_files || !file_blocks || !size || !counts || !file_ms || !file_depths || !coef || !J || !labels)
    return fail(LZ_E_INVAL, "null argument");
  if (fixed >= kSelTuples) return fail(LZ_E_INVAL, "fixed tuple index out of range");
  const uint32_t T = kSelTuples;
  // whole-file rows: token, match and match-byte totals, depths, 1
  std::vector<uint64_t> first(n_files + 1, 0);
  for (uint32_t f = 0; f < n_files; ++f) {
    if (!file_blocks[f]) return fail(LZ_E_INVAL, "file %u has no blocks", f);
    first[f + 1] = first[f] + file_blocks[f];
  }
  double A[25] = {0}, b[5] = {0};
  for (uint32_t f = 0; f < n_files; ++f)
    for (uint32_t t = 0; t < T; ++t) {
      double row[5] = {0, 0, 0, double(file_depths[f * T + t]), 1.0};
      for (uint64_t k = first[f]; k < first[f + 1]; ++k)
        for (int c = 0; c < 3; ++c) row[c] += double(counts[(k * T + t) * 3 + c]);
      for (int i = 0; i < 5; ++i) {
        b[i] += row[i] * file_ms[f * T + t];
        for (int j = 0; j < 5; ++j) A[i * 5 + j] += row[i] * row[j];
      }
    }
  // normal equations, columns scaled to unit diagonal for conditioning
  double sc[5];
  for (int i = 0; i < 5; ++i) sc[i] = A[i * 5 + i] > 0 ? 1.0 / sqrt(A[i * 5 + i]) : 1.0;
  for (int i = 0; i < 5; ++i) {
    b[i] *= sc[i];
    for (int j = 0; j < 5; ++j) A[i * 5 + j] *= sc[i] * sc[j];
  }
  double c[5];
  solve_small(5, A, b, c);
  for (int i = 0; i < 5; ++i) coef[i] = std::max(0.0, c[i] * sc[i]);
  // per-block cost against the fixed tuple, and its minimiser
  for (uint32_t f = 0; f < n_files; ++f)
    for (uint64_t k = first[f]; k < first[f + 1]; ++k) {
      double tm[kSelTuples];
      for (uint32_t t = 0; t < T; ++t) {
        const uint64_t* q = counts + (k * T + t) * 3;
        const double v = coef[0] * q[0] + coef[1] * q[1] + coef[2] * q[2] +
                         (coef[3] * file_depths[f * T + t] + coef[4]) / file_blocks[f];
        tm[t] = std::max(v, 1e-12);
      }
      int32_t best = 0;
      for (uint32_t t = 0; t < T; ++t) {
        const double sf = size[k * T + fixed];
        J[k * T + t] = (sf > 0 ? size[k * T + t] / sf : 1.0) + lambda * tm[t] / tm[fixed];
        if (J[k * T + t] < J[k * T + best]) best = (int32_t)t;
      }
      labels[k] = best;
    }
  return 0;
}

int lz_selector_choose(const lz_selector* s, const float* feats, uint64_t n_rows, uint8_t* choice, float* top_prob) {
  if (!s || (n_rows && (!feats || !choice))) return fail(LZ_E_INVAL, "null argument");
  for (uint64_t r = 0; r < n_rows; ++r) {
    double p[kSelTuples];
    forward_row(s, feats + r * kSelIn, p);
    const uint32_t k = argmax16(p);
    // fallback: the fixed tuple unless the network is sure and the tuple
    // beat the fixed one on the validation blocks it was predicted for
    const bool ok = p[k] >= 0.5 && s->val_J[k] < 1.f;
    choice[r] = (uint8_t)(ok ? k : s->fixed);
    if (top_prob) top_prob[r] = (float)p[k];
  }
  return 0;
}

int lz_selector_calibrate(lz_selector* s, const float* feats, const double* J, uint64_t n_rows, double lambda) {
  if (!s || (n_rows && (!feats || !J))) return fail(LZ_E_INVAL, "null argument");
  double sum[kSelTuples] = {0};
  uint64_t cnt[kSelTuples] = {0};
  for (uint64_t r = 0; r < n_rows; ++r) {
    double p[kSelTuples];
    forward_row(s, feats + r * kSelIn, p);
    const uint32_t k = argmax16(p);
    sum[k] += J[r * kSelTuples + k];
    ++cnt[k];
  }
  // mean cost of a predicted tuple relative to the fixed tuple's (1 + lambda);
  // tuples never predicted are never trusted
  for (uint32_t t = 0; t < kSelTuples; ++t) s->val_J[t] = cnt[t] ? float(sum[t] / cnt[t] / (1.0 + lambda)) : 9.f;
  s->val_J[s->fixed] = 1.f;
  return 0;
}

int lz_selector_set_norm(lz_selector* s, const float* feats, uint64_t n_rows) {
  if (!s || (n_rows && !feats)) return fail(LZ_E_INVAL, "null argument");
  for (uint32_t i = 0; i < kSelIn; ++i) {
    double m = 0, v = 0;
    for (uint64_t r = 0; r < n_rows; ++r) m += feats[r * kSelIn + i];
    m = n_rows ? m / n_rows : 0;
    for (uint64_t r = 0; r < n_rows; ++r) {
      const double d = feats[r * kSelIn + i] - m;
      v += d * d;
    }
    v = n_rows ? v / n_rows : 0;
    s->mu[i] = float(m);
    s->sd[i] = float(sqrt(v) + 1e-6);
  }
  return 0;
}

int lz_encode_learned(const uint8_t* in, uint64_t n, const lz_params* p, const lz_selector* s, uint8_t** arc,
                      uint64_t* arc_size, uint8_t* choice) {
  if (!p || !s || !arc || !arc_size || (n && !in)) return fail(LZ_E_INVAL, "null argument");
  // features from a cheap parse: thresholds 4/4/4/4, 16 candidates per chain,
  // nearest source on ties
  lz_params q = *p;
  for (int k = 0; k < 4; ++k) q.thr[k] = 4;
  q.max_chain = 16;
  q.depth_passes = 0;
  q.progress = nullptr;
  uint8_t* cheap = nullptr;
  uint64_t cheap_size = 0;
  int rc = lz_encode(in, n, &q, &cheap, &cheap_size);
  if (rc) return rc;
  const uint64_t bs = 1ull << p->log2_bs, nb = (n + bs - 1) / bs;
  std::vector<float> feats(nb * kSelIn);
  std::vector<uint8_t> pick(nb);
  rc = nb ? lz_block_features(cheap, cheap_size, p->bound, feats.data()) : 0;
  lz_free(cheap);
  if (rc) return rc;
  rc = lz_selector_choose(s, feats.data(), nb, pick.data(), nullptr);
  if (rc) return rc;
  std::vector<uint32_t> thr(4 * nb);
  for (uint64_t b = 0; b < nb; ++b)
    for (int k = 0; k < 4; ++k) thr[4 * b + k] = s->tuples[pick[b]][k];
  if (choice) memcpy(choice, pick.data(), nb);
  return lz_encode_blockwise(in, n, p, thr.data(), pick.data(), arc, arc_size);
}

}  // extern "C"
