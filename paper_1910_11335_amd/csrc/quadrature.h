// Host-side level-symmetric quadrature of the library.
#pragma once
#include <string>
#include <vector>

namespace dsn {

bool lqn_supported(int N);

// omega: [N(N+2)][3], w: [N(N+2)] (sum 4 pi); order n = o*D + p with octant o
// and the point p of octant 0 reflected by the signs of o.
bool lqn_build(int N, std::vector<double> &omega, std::vector<double> &w, std::string &err);

}  // namespace dsn
