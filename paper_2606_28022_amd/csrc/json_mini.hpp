// Minimal JSON reader for the parameter file (objects, arrays, numbers,
// strings, true/false/null).  Parsing errors throw std::runtime_error, which
// the C ABI turns into an error code.
#pragma once

#include <cctype>
#include <cstdlib>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

namespace fx {

struct JVal {
  enum Kind { NUL, BOOL, NUM, STR, ARR, OBJ } kind = NUL;
  double num = 0.0;
  bool b = false;
  std::string str;
  std::vector<JVal> arr;
  std::map<std::string, JVal> obj;

  const JVal& operator[](const std::string& k) const {
    auto it = obj.find(k);
    if (kind != OBJ || it == obj.end()) throw std::runtime_error("json: missing key '" + k + "'");
    return it->second;
  }
  const JVal& operator[](size_t i) const {
    if (kind != ARR || i >= arr.size()) throw std::runtime_error("json: bad array index");
    return arr[i];
  }
  bool has(const std::string& k) const { return kind == OBJ && obj.count(k); }
  double d() const {
    if (kind != NUM) throw std::runtime_error("json: number expected");
    return num;
  }
  int i() const { return static_cast<int>(d()); }
  size_t size() const { return kind == ARR ? arr.size() : obj.size(); }
};

class JParser {
 public:
  explicit JParser(const std::string& s) : s_(s) {}
  JVal parse() {
    JVal v = value();
    ws();
    if (p_ != s_.size()) throw std::runtime_error("json: trailing characters");
    return v;
  }

 private:
  const std::string& s_;
  size_t p_ = 0;
  void ws() {
    while (p_ < s_.size() && std::isspace(static_cast<unsigned char>(s_[p_]))) ++p_;
  }
  char peek() {
    ws();
    if (p_ >= s_.size()) throw std::runtime_error("json: unexpected end");
    return s_[p_];
  }
  void expect(char c) {
    if (peek() != c) throw std::runtime_error(std::string("json: expected '") + c + "'");
    ++p_;
  }
  JVal value() {
    char c = peek();
    if (c == '{') return object();
    if (c == '[') return array();
    if (c == '"') {
      JVal v;
      v.kind = JVal::STR;
      v.str = string();
      return v;
    }
    if (s_.compare(p_, 4, "true") == 0) { p_ += 4; JVal v; v.kind = JVal::BOOL; v.b = true; return v; }
    if (s_.compare(p_, 5, "false") == 0) { p_ += 5; JVal v; v.kind = JVal::BOOL; return v; }
    if (s_.compare(p_, 4, "null") == 0) { p_ += 4; return JVal(); }
    return number();
  }
  std::string string() {
    expect('"');
    std::string out;
    while (p_ < s_.size() && s_[p_] != '"') {
      if (s_[p_] == '\\') {
        ++p_;
        if (p_ >= s_.size()) break;
        char e = s_[p_];
        out += (e == 'n') ? '\n' : (e == 't') ? '\t' : e;
      } else {
        out += s_[p_];
      }
      ++p_;
    }
    if (p_ >= s_.size()) throw std::runtime_error("json: unterminated string");
    ++p_;
    return out;
  }
  JVal number() {
    ws();
    const char* b = s_.c_str() + p_;
    char* e = nullptr;
    double x = std::strtod(b, &e);
    if (e == b) throw std::runtime_error("json: bad value");
    p_ += static_cast<size_t>(e - b);
    JVal v;
    v.kind = JVal::NUM;
    v.num = x;
    return v;
  }
  JVal array() {
    expect('[');
    JVal v;
    v.kind = JVal::ARR;
    if (peek() == ']') { ++p_; return v; }
    for (;;) {
      v.arr.push_back(value());
      char c = peek();
      ++p_;
      if (c == ']') break;
      if (c != ',') throw std::runtime_error("json: expected ',' in array");
    }
    return v;
  }
  JVal object() {
    expect('{');
    JVal v;
    v.kind = JVal::OBJ;
    if (peek() == '}') { ++p_; return v; }
    for (;;) {
      std::string k = string();
      expect(':');
      v.obj[k] = value();
      char c = peek();
      ++p_;
      if (c == '}') break;
      if (c != ',') throw std::runtime_error("json: expected ',' in object");
    }
    return v;
  }
};

}  // namespace fx
