// Minimal JSON reader for mechanism files (objects, arrays, strings, numbers, true/false/null).
// Numbers are parsed with strtod, which rounds correctly, so a file written with round-trip
// float formatting yields the exact same doubles on every reader.
#pragma once

#include <cstdlib>
#include <map>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

namespace chemjson {

struct Value {
  enum Kind { Null, Bool, Number, String, Array, Object } kind = Null;
  bool b = false;
  double num = 0.0;
  std::string str;
  std::vector<Value> arr;
  std::vector<std::pair<std::string, Value>> obj;  // keeps file order

  bool has(const std::string& k) const {
    if (kind != Object) return false;
    for (auto& kv : obj)
      if (kv.first == k) return true;
    return false;
  }
  const Value& operator[](const std::string& k) const {
    if (kind != Object) throw std::runtime_error("expected object when looking up '" + k + "'");
    for (auto& kv : obj)
      if (kv.first == k) return kv.second;
    throw std::runtime_error("missing key '" + k + "'");
  }
  const Value& operator[](size_t i) const {
    if (kind != Array || i >= arr.size()) throw std::runtime_error("array index out of range");
    return arr[i];
  }
  double number() const {
    if (kind != Number) throw std::runtime_error("expected a number");
    return num;
  }
  const std::string& string() const {
    if (kind != String) throw std::runtime_error("expected a string");
    return str;
  }
  size_t size() const { return kind == Array ? arr.size() : (kind == Object ? obj.size() : 0); }
};

class Parser {
 public:
  explicit Parser(const std::string& text) : s_(text) {}
  Value parse() {
    Value v = value();
    ws();
    if (i_ != s_.size()) fail("trailing characters");
    return v;
  }

 private:
  const std::string& s_;
  size_t i_ = 0;

  [[noreturn]] void fail(const char* what) {
    throw std::runtime_error(std::string("JSON parse error: ") + what + " at offset " + std::to_string(i_));
  }
  void ws() {
    while (i_ < s_.size() && (s_[i_] == ' ' || s_[i_] == '\n' || s_[i_] == '\t' || s_[i_] == '\r')) ++i_;
  }
  char peek() {
    ws();
    if (i_ >= s_.size()) fail("unexpected end");
    return s_[i_];
  }
  void expect(char c) {
    if (peek() != c) fail("unexpected character");
    ++i_;
  }
  Value value() {
    char c = peek();
    if (c == '{') return object();
    if (c == '[') return array();
    if (c == '"') {
      Value v;
      v.kind = Value::String;
      v.str = string();
      return v;
    }
    if (s_.compare(i_, 4, "true") == 0) { i_ += 4; Value v; v.kind = Value::Bool; v.b = true; return v; }
    if (s_.compare(i_, 5, "false") == 0) { i_ += 5; Value v; v.kind = Value::Bool; return v; }
    if (s_.compare(i_, 4, "null") == 0) { i_ += 4; return Value(); }
    return number();
  }
  Value number() {
    const char* start = s_.c_str() + i_;
    char* end = nullptr;
    double d = std::strtod(start, &end);
    if (end == start) fail("bad number");
    i_ += static_cast<size_t>(end - start);
    Value v;
    v.kind = Value::Number;
    v.num = d;
    return v;
  }
  std::string string() {
    expect('"');
    std::string out;
    while (i_ < s_.size() && s_[i_] != '"') {
      char c = s_[i_++];
      if (c == '\\') {
        if (i_ >= s_.size()) fail("bad escape");
        char e = s_[i_++];
        switch (e) {
          case 'n': out += '\n'; break;
          case 't': out += '\t'; break;
          case 'r': out += '\r'; break;
          case 'b': out += '\b'; break;
          case 'f': out += '\f'; break;
          case 'u': {  // keep ASCII, replace the rest
            if (i_ + 4 > s_.size()) fail("bad \\u escape");
            unsigned code = static_cast<unsigned>(std::strtoul(s_.substr(i_, 4).c_str(), nullptr, 16));
            i_ += 4;
            out += code < 128 ? static_cast<char>(code) : '?';
            break;
          }
          default: out += e;
        }
      } else {
        out += c;
      }
    }
    if (i_ >= s_.size()) fail("unterminated string");
    ++i_;
    return out;
  }
  Value array() {
    expect('[');
    Value v;
    v.kind = Value::Array;
    if (peek() == ']') { ++i_; return v; }
    while (true) {
      v.arr.push_back(value());
      char c = peek();
      ++i_;
      if (c == ']') break;
      if (c != ',') fail("expected , or ]");
    }
    return v;
  }
  Value object() {
    expect('{');
    Value v;
    v.kind = Value::Object;
    if (peek() == '}') { ++i_; return v; }
    while (true) {
      if (peek() != '"') fail("expected key");
      std::string k = string();
      expect(':');
      v.obj.emplace_back(k, value());
      char c = peek();
      ++i_;
      if (c == '}') break;
      if (c != ',') fail("expected , or }");
    }
    return v;
  }
};

inline Value parse(const std::string& text) { return Parser(text).parse(); }

}  // namespace chemjson
