// N-Triples dictionary encoder (Section 6.2.1, step 2): RDF text in, integer
// triples out, with the dictionaries kept for decoding. Subjects and objects
// share one dictionary numbered from 0, predicates have their own numbered
// from 1, each in order of first appearance (lines in order, a line's subject
// before its object). A term is keyed by its bytes as written (an IRI with its
// angle brackets, "_:label", a literal with its quotes, escapes and language
// tag or datatype). Host code: one pass over the text, hash maps over views of
// a private copy of it.
#include <algorithm>
#include <climits>
#include <cstring>
#include <new>
#include <string>
#include <string_view>
#include <unordered_map>
#include <vector>

#include "gsmart.h"

namespace gs {
void set_error(const std::string &msg);
}
using gs::set_error;

struct gs_dict {
  std::string text;   // private copy: every term is a view into it
  std::unordered_map<std::string_view, int64_t> vid;
  std::unordered_map<std::string_view, int32_t> pid;
  std::vector<std::string_view> vertices, labels;   // labels[k] is predicate k + 1
  std::vector<int32_t> triples;                     // 3 per line
};

namespace {

bool ascii_alnum(char c) { return (c >= 'a' && c <= 'z') || (c >= 'A' && c <= 'Z') || (c >= '0' && c <= '9'); }

// The term that starts at p (no leading blank), up to e. Returns its end, or nullptr with msg set.
const char *term_end(const char *p, const char *e, const char *&msg) {
  if (*p == '<') {
    const char *q = static_cast<const char *>(memchr(p + 1, '>', (size_t)(e - p - 1)));
    if (!q) { msg = "unterminated IRI"; return nullptr; }
    return q + 1;
  }
  if (e - p >= 2 && p[0] == '_' && p[1] == ':') {
    const char *q = p + 2;
    while (q < e && (ascii_alnum(*q) || *q == '_' || *q == '-')) ++q;
    if (q == p + 2) { msg = "empty blank node label"; return nullptr; }
    return q;
  }
  if (*p == '"') {
    const char *q = p + 1;
    for (;;) {
      if (q >= e) { msg = "unterminated literal"; return nullptr; }
      if (*q == '\\') { q += 2; continue; }
      if (*q == '"') break;
      ++q;
    }
    ++q;
    if (q < e && *q == '@') {
      ++q;
      while (q < e && (ascii_alnum(*q) || *q == '-')) ++q;
    } else if (e - q >= 3 && q[0] == '^' && q[1] == '^' && q[2] == '<') {
      const char *r = static_cast<const char *>(memchr(q + 3, '>', (size_t)(e - q - 3)));
      if (!r) { msg = "unterminated datatype IRI"; return nullptr; }
      q = r + 1;
    }
    return q;
  }
  msg = "a term starts with <, _: or a quote";
  return nullptr;
}

}  // namespace

extern "C" {

gs_status gs_encode_ntriples(const char *text, int64_t len, gs_dict **out) {
  if (!out || (!text && len > 0) || len < 0) { set_error("gs_encode_ntriples: bad arguments"); return GS_EINVAL; }
  *out = nullptr;
  gs_dict *d = new (std::nothrow) gs_dict;
  if (!d) { set_error("out of host memory"); return GS_ENOMEM; }
  try {
    d->text.assign(text, (size_t)len);
    const char *p = d->text.data(), *end = p + d->text.size();
    int64_t line = 0;
    while (p < end) {
      ++line;
      const char *nl = static_cast<const char *>(memchr(p, '\n', (size_t)(end - p)));
      const char *e = nl ? nl : end;
      const char *next = nl ? nl + 1 : end;
      if (e > p && e[-1] == '\r') --e;
      auto skip = [&](const char *q) { while (q < e && (*q == ' ' || *q == '\t')) ++q; return q; };
      const char *q = skip(p);
      if (q == e || *q == '#') { p = next; continue; }
      std::string_view t[3];
      const char *msg = nullptr;
      for (int k = 0; k < 3; ++k) {
        if (q == e) { msg = "fewer than three terms"; break; }
        const char *r = term_end(q, e, msg);
        if (!r) break;
        t[k] = std::string_view(q, (size_t)(r - q));
        q = skip(r);
      }
      if (!msg && (q == e || *q != '.')) msg = "a triple ends with '.'";
      if (!msg) {
        q = skip(q + 1);
        if (q < e && *q != '#') msg = "text after the final '.'";
      }
      if (!msg && t[0][0] == '"') msg = "a literal cannot be a subject";
      if (!msg && t[1][0] != '<') msg = "a predicate is an IRI";
      if (msg) {
        set_error("N-Triples line " + std::to_string(line) + ": " + msg);
        delete d;
        return GS_EINVAL;
      }
      int64_t ids[2];
      for (int k = 0; k < 2; ++k) {
        const std::string_view v = t[k == 0 ? 0 : 2];
        auto it = d->vid.find(v);
        if (it == d->vid.end()) {
          it = d->vid.emplace(v, (int64_t)d->vertices.size()).first;
          d->vertices.push_back(v);
        }
        ids[k] = it->second;
      }
      auto pt = d->pid.find(t[1]);
      if (pt == d->pid.end()) {
        pt = d->pid.emplace(t[1], (int32_t)d->labels.size() + 1).first;
        d->labels.push_back(t[1]);
      }
      if (ids[0] > INT32_MAX || ids[1] > INT32_MAX) {
        set_error("more than 2^31 distinct subjects and objects");
        delete d;
        return GS_ERANGE;
      }
      d->triples.push_back((int32_t)ids[0]);
      d->triples.push_back(pt->second);
      d->triples.push_back((int32_t)ids[1]);
      p = next;
    }
  } catch (const std::bad_alloc &) {
    delete d;
    set_error("out of host memory");
    return GS_ENOMEM;
  }
  *out = d;
  return GS_OK;
}

gs_status gs_dict_info(const gs_dict *d, int64_t *n_triples, int64_t *n_vertices, int32_t *n_labels) {
  if (!d) { set_error("null dictionary"); return GS_EINVAL; }
  if (n_triples) *n_triples = (int64_t)d->triples.size() / 3;
  if (n_vertices) *n_vertices = (int64_t)d->vertices.size();
  if (n_labels) *n_labels = (int32_t)d->labels.size();
  return GS_OK;
}

gs_status gs_dict_triples(const gs_dict *d, int32_t *out) {
  if (!d || (!out && !d->triples.empty())) { set_error("gs_dict_triples: bad arguments"); return GS_EINVAL; }
  if (!d->triples.empty()) memcpy(out, d->triples.data(), sizeof(int32_t) * d->triples.size());
  return GS_OK;
}

static gs_status copy_term(std::string_view v, char *buf, int64_t cap, int64_t *len) {
  if (len) *len = (int64_t)v.size();
  if (buf && cap > 0) {
    const size_t n = std::min<size_t>(v.size(), (size_t)cap - 1);
    memcpy(buf, v.data(), n);
    buf[n] = 0;
  }
  return GS_OK;
}

gs_status gs_dict_vertex(const gs_dict *d, int64_t id, char *buf, int64_t cap, int64_t *len) {
  if (!d || id < 0 || id >= (int64_t)d->vertices.size()) { set_error("vertex id out of range"); return GS_ERANGE; }
  return copy_term(d->vertices[(size_t)id], buf, cap, len);
}

gs_status gs_dict_label(const gs_dict *d, int32_t label, char *buf, int64_t cap, int64_t *len) {
  if (!d || label < 1 || label > (int32_t)d->labels.size()) { set_error("label out of range"); return GS_ERANGE; }
  return copy_term(d->labels[(size_t)label - 1], buf, cap, len);
}

gs_status gs_dict_find_vertex(const gs_dict *d, const char *term, int64_t len, int64_t *id) {
  if (!d || !id || (!term && len > 0)) { set_error("gs_dict_find_vertex: bad arguments"); return GS_EINVAL; }
  auto it = d->vid.find(std::string_view(term, (size_t)len));
  *id = it == d->vid.end() ? -1 : it->second;
  return GS_OK;
}

gs_status gs_dict_find_label(const gs_dict *d, const char *term, int64_t len, int32_t *label) {
  if (!d || !label || (!term && len > 0)) { set_error("gs_dict_find_label: bad arguments"); return GS_EINVAL; }
  auto it = d->pid.find(std::string_view(term, (size_t)len));
  *label = it == d->pid.end() ? 0 : it->second;
  return GS_OK;
}

gs_status gs_dict_free(gs_dict *d) {
  delete d;
  return GS_OK;
}

}  // extern "C"
