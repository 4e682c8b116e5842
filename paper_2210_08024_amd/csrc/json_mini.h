// Minimal JSON reader (host only) for the coefficient file: objects, arrays,
// numbers, strings, true/false/null.  Enough for a data file we write ourselves.
#pragma once
#include <cctype>
#include <cstdlib>
#include <map>
#include <memory>
#include <string>
#include <vector>

namespace ismjson {

struct Value {
  enum Kind { Null, Bool, Num, Str, Arr, Obj } kind = Null;
  double num = 0.0;
  bool b = false;
  std::string str;
  std::vector<Value> arr;
  std::map<std::string, Value> obj;

  const Value *get(const std::string &k) const {
    if (kind != Obj) return nullptr;
    auto it = obj.find(k);
    return it == obj.end() ? nullptr : &it->second;
  }
  // Flatten a number or (nested) array of numbers.
  bool numbers(std::vector<double> &out) const {
    if (kind == Num) { out.push_back(num); return true; }
    if (kind != Arr) return false;
    for (const auto &v : arr)
      if (!v.numbers(out)) return false;
    return true;
  }
};

class Parser {
 public:
  explicit Parser(const std::string &s) : s_(s) {}
  bool parse(Value &v, std::string &err) {
    pos_ = 0;
    if (!value(v)) { err = "JSON parse error near offset " + std::to_string(pos_); return false; }
    ws();
    if (pos_ != s_.size()) { err = "trailing data at offset " + std::to_string(pos_); return false; }
    return true;
  }

 private:
  const std::string &s_;
  size_t pos_ = 0;
  void ws() { while (pos_ < s_.size() && std::isspace((unsigned char)s_[pos_])) ++pos_; }
  bool lit(const char *w) {
    size_t n = std::char_traits<char>::length(w);
    if (s_.compare(pos_, n, w) != 0) return false;
    pos_ += n;
    return true;
  }
  bool string(std::string &out) {
    if (pos_ >= s_.size() || s_[pos_] != '"') return false;
    ++pos_;
    while (pos_ < s_.size() && s_[pos_] != '"') {
      char c = s_[pos_++];
      if (c == '\\') {
        if (pos_ >= s_.size()) return false;
        char e = s_[pos_++];
        switch (e) {
          case 'n': out += '\n'; break;
          case 't': out += '\t'; break;
          case 'u': pos_ += 4; out += '?'; break;  // non-ASCII escapes are not needed here
          default: out += e;
        }
      } else {
        out += c;
      }
    }
    if (pos_ >= s_.size()) return false;
    ++pos_;
    return true;
  }
  bool value(Value &v) {
    ws();
    if (pos_ >= s_.size()) return false;
    char c = s_[pos_];
    if (c == '{') {
      v.kind = Value::Obj;
      ++pos_;
      ws();
      if (pos_ < s_.size() && s_[pos_] == '}') { ++pos_; return true; }
      for (;;) {
        ws();
        std::string k;
        if (!string(k)) return false;
        ws();
        if (pos_ >= s_.size() || s_[pos_] != ':') return false;
        ++pos_;
        if (!value(v.obj[k])) return false;
        ws();
        if (pos_ < s_.size() && s_[pos_] == ',') { ++pos_; continue; }
        if (pos_ < s_.size() && s_[pos_] == '}') { ++pos_; return true; }
        return false;
      }
    }
    if (c == '[') {
      v.kind = Value::Arr;
      ++pos_;
      ws();
      if (pos_ < s_.size() && s_[pos_] == ']') { ++pos_; return true; }
      for (;;) {
        v.arr.emplace_back();
        if (!value(v.arr.back())) return false;
        ws();
        if (pos_ < s_.size() && s_[pos_] == ',') { ++pos_; continue; }
        if (pos_ < s_.size() && s_[pos_] == ']') { ++pos_; return true; }
        return false;
      }
    }
    if (c == '"') { v.kind = Value::Str; return string(v.str); }
    if (lit("true")) { v.kind = Value::Bool; v.b = true; return true; }
    if (lit("false")) { v.kind = Value::Bool; v.b = false; return true; }
    if (lit("null")) { v.kind = Value::Null; return true; }
    const char *b = s_.c_str() + pos_;
    char *e = nullptr;
    double d = std::strtod(b, &e);
    if (e == b) return false;
    pos_ += (size_t)(e - b);
    v.kind = Value::Num;
    v.num = d;
    return true;
  }
};

}  // namespace ismjson
