// Prints the generated HIP source of a mechanism file (for the CPU emulation test).
#include <fstream>
#include <iostream>
#include <sstream>

#include "mechanism.hpp"

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  std::ifstream f(argv[1]);
  std::stringstream ss;
  ss << f.rdbuf();
  std::cout << chem::generate_source(chem::parse_mechanism(ss.str()), 24);
  return 0;
}
