// Range-partitioned contraction with re-issue of failed ranges and a JSONL
// checkpoint of completed ones.
//
// The slices of a cut network are independent and identical in cost, and the
// master only sums one value per slice (Sec. III A); a lost part of the work
// is recovered by contracting the missing slices again (Sec. V).  Here the
// slice space [0, 2^k) is split into fixed ranges; each range is one
// qtn_contract call, a failed call is issued again, completed ranges are
// appended to a checkpoint file, and the range partials are combined with
// TwoSum in ascending range order, so the amplitude is the same bit for bit
// whichever ranges were re-issued or resumed.
#include <cerrno>
#include <cinttypes>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <unistd.h>
#include <vector>

#include "../../include/qtn.h"
#include "plan_state.h"

namespace qtn {

// FNV-1a over the data that defines the plan's amplitudes and slices.
static uint64_t fingerprint(const qtn_plan_t *P) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&](const void *p, size_t n) {
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < n; ++i) {
      h ^= c[i];
      h *= 1099511628211ull;
    }
  };
  const Network &N = P->net;
  mix(&N.n, sizeof N.n);
  mix(&N.p, sizeof N.p);
  mix(&N.B, sizeof N.B);
  for (const auto &e : N.edges) {
    mix(&e.first, sizeof e.first);
    mix(&e.second, sizeof e.second);
  }
  mix(N.gamma.data(), N.gamma.size() * sizeof(double));
  mix(N.beta.data(), N.beta.size() * sizeof(double));
  mix(N.bits.data(), N.bits.size());
  for (const auto &v : N.values) mix(v.data(), v.size() * sizeof(cd));   // every gate tensor
  for (int c : P->cut) mix(&c, sizeof c);
  mix(&P->precision, sizeof P->precision);
  return h;
}

static std::string header_line(uint64_t fp, uint64_t R, uint32_t B, uint32_t k) {
  char buf[256];
  std::snprintf(buf, sizeof buf,
                "{\"qtn_checkpoint\": 1, \"plan\": \"%016" PRIx64 "\", \"range_slices\": %" PRIu64
                ", \"bitstrings\": %u, \"k\": %u}",
                fp, R, B, k);
  return buf;
}

// One completed range: {"lo": L, "hi": H, "p": ["<hex>", ...]} with four
// hexadecimal doubles (re, im, re_comp, im_comp) per bitstring.
static std::string range_line(uint64_t lo, uint64_t hi, const std::vector<qtn_partial> &p) {
  std::string s = "{\"lo\": " + std::to_string(lo) + ", \"hi\": " + std::to_string(hi) + ", \"p\": [";
  char buf[64];
  for (size_t b = 0; b < p.size(); ++b) {
    const double v[4] = {p[b].re, p[b].im, p[b].re_comp, p[b].im_comp};
    for (int j = 0; j < 4; ++j) {
      std::snprintf(buf, sizeof buf, "%s\"%a\"", (b || j) ? ", " : "", v[j]);
      s += buf;
    }
  }
  return s + "]}";
}

// Parses a range line; false for anything malformed (a torn last line).
static bool parse_range(const std::string &line, uint32_t B, uint64_t &lo, uint64_t &hi,
                        std::vector<qtn_partial> &p) {
  if (std::sscanf(line.c_str(), "{\"lo\": %" SCNu64 ", \"hi\": %" SCNu64 ",", &lo, &hi) != 2) return false;
  size_t at = line.find("\"p\": [");
  if (at == std::string::npos) return false;
  at += 6;
  std::vector<double> v;
  while (v.size() < 4ull * B) {
    const size_t q0 = line.find('"', at);
    if (q0 == std::string::npos) return false;
    const size_t q1 = line.find('"', q0 + 1);
    if (q1 == std::string::npos) return false;
    const std::string tok = line.substr(q0 + 1, q1 - q0 - 1);
    char *end = nullptr;
    errno = 0;
    const double d = std::strtod(tok.c_str(), &end);
    if (errno || !end || *end) return false;
    v.push_back(d);
    at = q1 + 1;
  }
  if (line.find("]}", at) == std::string::npos) return false;
  p.resize(B);
  for (uint32_t b = 0; b < B; ++b) p[b] = qtn_partial{v[4 * b], v[4 * b + 1], v[4 * b + 2], v[4 * b + 3]};
  return true;
}

}  // namespace qtn

using namespace qtn;

extern "C" int qtn_plan_fingerprint(const qtn_plan_t *P, uint64_t *out) {
  if (!P || !out) {
    set_error("NULL argument");
    return QTN_EINVAL;
  }
  *out = fingerprint(P);
  return QTN_OK;
}

extern "C" int qtn_plan_inject_faults(qtn_plan_t *P, uint64_t slice_lo, int32_t count) {
  if (!P || count < 0) {
    set_error("NULL plan or negative count");
    return QTN_EINVAL;
  }
  P->fault_lo = slice_lo;
  P->fault_count = count;
  return QTN_OK;
}

extern "C" int qtn_contract_ranges(qtn_plan_t *P, uint64_t range_slices, int32_t max_retries,
                                   const char *checkpoint, void *stream, qtn_partial *out,
                                   qtn_range_stats *stats) {
  set_error("");
  if (!P || !out) {
    set_error("NULL argument");
    return QTN_EINVAL;
  }
  if (range_slices == 0 || max_retries < 0) {
    set_error("range_slices must be >= 1 and max_retries >= 0");
    return QTN_EINVAL;
  }
  const uint64_t total = 1ull << P->cut.size();
  const uint32_t B = P->net.B;
  const uint64_t nr = (total + range_slices - 1) / range_slices;
  if (nr > (1ull << 26)) {
    set_error("too many ranges (at most 2^26)");
    return QTN_EINVAL;
  }
  qtn_range_stats st;
  std::memset(&st, 0, sizeof st);
  st.ranges = nr;
  std::vector<std::vector<qtn_partial>> part(nr);
  std::vector<char> done(nr, 0);
  const uint64_t fp = fingerprint(P);
  const std::string head = header_line(fp, range_slices, B, (uint32_t)P->cut.size());
  FILE *ck = nullptr;
  if (checkpoint && checkpoint[0]) {
    // resume: every well-formed line of a checkpoint of this plan and range
    // size is a completed range; a torn last line is ignored and rewritten
    std::vector<std::string> keep;
    if (FILE *f = std::fopen(checkpoint, "r")) {
      std::string line;
      bool first = true;
      int c;
      auto take = [&](const std::string &l) -> int {
        if (first) {
          first = false;
          if (l != head) {
            set_error("checkpoint " + std::string(checkpoint) +
                      " belongs to another plan or range size");
            return QTN_EINVAL;
          }
          keep.push_back(l);
          return QTN_OK;
        }
        uint64_t lo, hi;
        std::vector<qtn_partial> p;
        if (!parse_range(l, B, lo, hi, p)) return QTN_OK;
        if (lo % range_slices || lo >= total || hi != std::min(total, lo + range_slices)) return QTN_OK;
        const uint64_t j = lo / range_slices;
        if (!done[j]) {
          done[j] = 1;
          part[j] = p;
          ++st.resumed;
          keep.push_back(l);
        }
        return QTN_OK;
      };
      int rc = QTN_OK;
      while (rc == QTN_OK && (c = std::fgetc(f)) != EOF) {
        if (c == '\n') {
          rc = take(line);
          line.clear();
        } else {
          line.push_back((char)c);
        }
      }
      std::fclose(f);
      if (rc != QTN_OK) return rc;
    }
    // rewrite the file with the header and the well-formed lines only
    const std::string tmp = std::string(checkpoint) + ".tmp";
    ck = std::fopen(tmp.c_str(), "w");
    if (!ck) {
      set_error("cannot write checkpoint " + tmp);
      return QTN_EINVAL;
    }
    if (keep.empty()) keep.push_back(head);
    for (const std::string &l : keep) std::fprintf(ck, "%s\n", l.c_str());
    std::fflush(ck);
    fsync(fileno(ck));
    std::fclose(ck);
    if (std::rename(tmp.c_str(), checkpoint) != 0) {
      set_error("cannot replace checkpoint " + std::string(checkpoint));
      return QTN_EINVAL;
    }
    ck = std::fopen(checkpoint, "a");
    if (!ck) {
      set_error("cannot append to checkpoint " + std::string(checkpoint));
      return QTN_EINVAL;
    }
  }
  int last_rc = QTN_OK;
  std::string last_msg;
  std::vector<qtn_partial> buf(B);
  for (int32_t round = 0; round <= max_retries; ++round) {
    bool failed = false;
    for (uint64_t j = 0; j < nr; ++j) {
      if (done[j]) continue;
      const uint64_t lo = j * range_slices, hi = std::min(total, lo + range_slices);
      int rc;
      if (P->fault_count > 0 && P->fault_lo == lo) {
        --P->fault_count;   // a fault forced from the host; no device work
        rc = QTN_EHIP;
        set_error("injected fault in range [" + std::to_string(lo) + ", " + std::to_string(hi) + ")");
      } else {
        rc = qtn_contract(P, lo, hi, stream, buf.data());
      }
      if (rc != QTN_OK) {
        failed = true;
        last_rc = rc;
        last_msg = qtn_last_error();
        if (round < max_retries) ++st.retried;
        if (rc == QTN_ETIMEOUT) break;  // work may still be in flight: stop here
        continue;
      }
      part[j] = buf;
      done[j] = 1;
      ++st.contracted;
      if (ck) {
        std::fprintf(ck, "%s\n", range_line(lo, hi, buf).c_str());
        std::fflush(ck);
        fsync(fileno(ck));
      }
    }
    if (!failed || last_rc == QTN_ETIMEOUT) break;
  }
  if (ck) std::fclose(ck);
  if (stats) *stats = st;
  for (uint64_t j = 0; j < nr; ++j)
    if (!done[j]) {
      set_error("range [" + std::to_string(j * range_slices) + ", ...) failed: " + last_msg);
      return last_rc;
    }
  // fixed combination order: ascending range start
  for (uint32_t b = 0; b < B; ++b) {
    qtn_partial acc = part[0][b];
    for (uint64_t j = 1; j < nr; ++j) qtn_partial_combine(&acc, &part[j][b], &acc);
    out[b] = acc;
  }
  return QTN_OK;
}
