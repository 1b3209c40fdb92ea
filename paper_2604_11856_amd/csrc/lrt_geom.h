// Host-only ray geometry of liblrt (Sec. 2.2.3): Gauss-Legendre polar
// nodes, the cell-to-cell traversal of an axisymmetric structured grid and
// the Fibonacci-sphere lines of sight with their angular rule.  Plain C++ with
// no device code, so it also builds on its own (sanitizer builds of the host
// geometry).  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace lrt {

// Message of the last failed call made without a context (this thread).
std::string &host_error();

// Gauss-Legendre nodes (ascending) and weights on [0, 1], weights summing to 1.
void gauss_legendre_01(int n, std::vector<double> &mu, std::vector<double> &w);

// Cell-to-cell traversal of one ray from the wall point (0, rw, 0) along
// (mu, st cos phi, st sin phi) through the nx x nr grid over [0, Lx] x
// [0, R]; appends (cell, path length) segments in wall -> far order.  Returns
// false if the traversal does not terminate.
bool traverse_axi(int nx, int nr, double Lx, double R, double rw, double mu, double phi,
                  std::vector<int32_t> &cell, std::vector<double> &ds);

// Fibonacci-sphere directions with a positive normal component (dir, 3 per
// direction, normal component first) and the flux weight of each.
void fibonacci_rule(int n_los, int n_polar, int n_azim, std::vector<double> &dir, std::vector<double> &wt);

}  // namespace lrt
