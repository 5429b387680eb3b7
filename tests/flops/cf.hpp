#pragma once
#include <cmath>
#include <cstdint>
// counting floating type: every + - * / on it counts one FLOP
static long long cnt_flop = 0, cnt_div = 0, cnt_rsqrt = 0, cnt_atan = 0, cnt_log = 0, cnt_sqrt = 0;
struct CF {
  double v;
  CF() : v(0) {}
  CF(double x) : v(x) {}
  static CF raw(double x) { CF c; c.v = x; return c; }
  explicit operator double() const { return v; }
  explicit operator float() const { return (float)v; }
  explicit operator int() const { return (int)v; }
};
inline CF operator+(CF a, CF b) { cnt_flop++; return CF::raw(a.v + b.v); }
inline CF operator-(CF a, CF b) { cnt_flop++; return CF::raw(a.v - b.v); }
inline CF operator*(CF a, CF b) { cnt_flop++; return CF::raw(a.v * b.v); }
inline CF operator/(CF a, CF b) { cnt_flop++; cnt_div++; return CF::raw(a.v / b.v); }
inline CF operator-(CF a) { return CF::raw(-a.v); }
inline CF& operator+=(CF& a, CF b) { a = a + b; return a; }
inline CF& operator-=(CF& a, CF b) { a = a - b; return a; }
inline CF& operator*=(CF& a, CF b) { a = a * b; return a; }
inline CF& operator/=(CF& a, CF b) { a = a / b; return a; }
inline bool operator<(CF a, CF b) { return a.v < b.v; }
inline bool operator>(CF a, CF b) { return a.v > b.v; }
inline bool operator<=(CF a, CF b) { return a.v <= b.v; }
inline bool operator>=(CF a, CF b) { return a.v >= b.v; }
inline bool operator==(CF a, CF b) { return a.v == b.v; }
inline bool operator!=(CF a, CF b) { return a.v != b.v; }
