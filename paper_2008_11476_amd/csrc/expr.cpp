// Recursive-descent parser of user point kernels into a postfix program.
//
//   sum     := product (('+' | '-') product)*
//   product := unary (('*' | '/') unary)*
//   unary   := '-' unary | primary
//   primary := number | 'a' | 'b' | 'c' | 'a' '[' offset ',' offset ']'
//            | name '(' sum (',' sum)* ')' | '(' sum ')'
//   offset  := ['-'] digit          (-2 .. 2; a local kernel's window read)
//
// Functions: min, max (2), abs (1), clamp (3), gt (2), sel (3), sqrt (1).
// The program keeps at most kExprStack values on its stack and holds at most
// kMaxExpr instructions and kMaxExprConst distinct literals.
#include "expr.h"

#include <cctype>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include <algorithm>

namespace hvx {

namespace {

struct Parser {
  const char* s;
  size_t i = 0;
  ExprProg* p;
  int depth = 0, max_depth = 0;
  std::string err;

  void ws() {
    while (s[i] == ' ' || s[i] == '\t' || s[i] == '\n' || s[i] == '\r') ++i;
  }
  bool fail(const std::string& m) {
    if (err.empty()) err = m + " at offset " + std::to_string(i);
    return false;
  }
  bool emit(int op, int arg, int pops, int pushes) {
    if ((int)p->code.size() >= kMaxExpr) return fail("expression longer than " + std::to_string(kMaxExpr) + " steps");
    p->code.push_back((int16_t)(op | (arg << 8)));
    depth += pushes - pops;
    if (depth > max_depth) max_depth = depth;
    if (max_depth > kExprStack) return fail("expression nests deeper than " + std::to_string(kExprStack) + " values");
    return true;
  }
  bool number() {
    const char* b = s + i;
    char* e = nullptr;
    double v = strtod(b, &e);
    if (e == b) return fail("number expected");
    // no hex floats, infinities or NaN spellings
    for (const char* q = b; q < e; ++q)
      if (!(isdigit((unsigned char)*q) || *q == '.' || *q == 'e' || *q == 'E' || *q == '+' || *q == '-'))
        return fail("malformed number");
    bool integral = true;
    for (const char* q = b; q < e; ++q) integral &= isdigit((unsigned char)*q) != 0;
    if (!integral) p->needs_float = true;
    if (integral && v > 2147483647.0) p->int_literals_ok = false;
    if (!std::isfinite(v)) return fail("literal out of range");
    i = (size_t)(e - s);
    int k = -1;
    for (size_t j = 0; j < p->consts.size(); ++j)
      if (p->consts[j] == v) k = (int)j;
    if (k < 0) {
      if ((int)p->consts.size() >= kMaxExprConst)
        return fail("more than " + std::to_string(kMaxExprConst) + " distinct literals");
      k = (int)p->consts.size();
      p->consts.push_back(v);
    }
    return emit(X_CONST, k, 0, 1);
  }
  bool primary() {
    ws();
    char ch = s[i];
    if (isdigit((unsigned char)ch) || ch == '.') return number();
    if (ch == '(') {
      ++i;
      if (!sum()) return false;
      ws();
      if (s[i] != ')') return fail("')' expected");
      ++i;
      return true;
    }
    if (!isalpha((unsigned char)ch)) return fail(ch ? "operand expected" : "unexpected end");
    size_t b = i;
    while (isalnum((unsigned char)s[i]) || s[i] == '_') ++i;
    std::string name(s + b, i - b);
    if (name == "a" || name == "b" || name == "c") {
      int k = name[0] - 'a';
      if (k > p->max_input) p->max_input = k;
      ws();
      if (s[i] != '[') return emit(X_IN, k, 0, 1);
      if (k != 0) return fail("offsets only on input a");
      ++i;
      int off[2];
      for (int j = 0; j < 2; ++j) {
        ws();
        bool neg = false;
        if (s[i] == '-') {
          neg = true;
          ++i;
          ws();
        }
        if (!isdigit((unsigned char)s[i]) || isdigit((unsigned char)s[i + 1])) return fail("offset must be one digit");
        off[j] = (s[i] - '0') * (neg ? -1 : 1);
        ++i;
        if (off[j] < -2 || off[j] > 2) return fail("offset outside -2..2");
        ws();
        if (s[i] != (j == 0 ? ',' : ']')) return fail(j == 0 ? "',' expected in a[dx, dy]" : "']' expected");
        ++i;
      }
      p->has_offsets = true;
      p->rx = std::max(p->rx, std::abs(off[0]));
      p->ry = std::max(p->ry, std::abs(off[1]));
      return emit(X_INW, (off[1] + 2) * 5 + (off[0] + 2), 0, 1);
    }
    struct F {
      const char* n;
      int op, args;
    };
    static const F fns[] = {{"min", X_MIN, 2}, {"max", X_MAX, 2}, {"abs", X_ABS, 1}, {"clamp", X_CLAMP, 3},
                            {"gt", X_GT, 2},   {"sel", X_SEL, 3}, {"sqrt", X_SQRT, 1}};
    const F* f = nullptr;
    for (const F& x : fns)
      if (name == x.n) f = &x;
    if (!f) return fail("unknown name '" + name + "'");
    if (f->op == X_SQRT) p->needs_float = true;
    ws();
    if (s[i] != '(') return fail("'(' expected after " + name);
    ++i;
    for (int k = 0; k < f->args; ++k) {
      if (k) {
        ws();
        if (s[i] != ',') return fail("',' expected in " + name);
        ++i;
      }
      if (!sum()) return false;
    }
    ws();
    if (s[i] != ')') return fail("')' expected after the arguments of " + name);
    ++i;
    return emit(f->op, 0, f->args, 1);
  }
  bool unary() {
    ws();
    if (s[i] == '-') {
      ++i;
      if (!unary()) return false;
      return emit(X_NEG, 0, 1, 1);
    }
    return primary();
  }
  bool product() {
    if (!unary()) return false;
    for (;;) {
      ws();
      char ch = s[i];
      if (ch != '*' && ch != '/') return true;
      ++i;
      if (!unary()) return false;
      if (!emit(ch == '*' ? X_MUL : X_DIV, 0, 2, 1)) return false;
    }
  }
  bool sum() {
    if (!product()) return false;
    for (;;) {
      ws();
      char ch = s[i];
      if (ch != '+' && ch != '-') return true;
      ++i;
      if (!product()) return false;
      if (!emit(ch == '+' ? X_ADD : X_SUB, 0, 2, 1)) return false;
    }
  }
};

}  // namespace

std::string parse_expr(const char* src, ExprProg* out) {
  *out = ExprProg{};
  if (!src) return "null expression";
  Parser ps{src, 0, out};
  if (!ps.sum()) return ps.err;
  ps.ws();
  if (src[ps.i] != '\0') {
    ps.fail("unexpected character");
    return ps.err;
  }
  return std::string();
}

}  // namespace hvx
