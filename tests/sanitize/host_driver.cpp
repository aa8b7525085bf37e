// Sanitizer driver for the library's host-side loader (no GPU calls): the
// mechanism parser on good and malformed texts, and the generated
// lane-per-cell source for both Newton-matrix modes.  Built with the host
// half under -fsanitize=address,undefined by tests/test_sanitizers.py.
#include "../../paper_2405_05974_amd/csrc/chem_host.cpp"
#include <fstream>
#include <iostream>
#include <sstream>

int main(int argc, char** argv) {
  if (argc < 2) return 2;
  std::ifstream f(argv[1]);
  std::stringstream ss;
  ss << f.rdbuf();
  chemgpu::HostMech hm;
  if (parse_mechanism(ss.str(), hm) != CHEM_OK) {
    std::cerr << "parse failed: " << g_last_error << "\n";
    return 1;
  }
  const std::string a = chemgpu::lpc_source(hm, false), b = chemgpu::lpc_source(hm, true);
  if (a.size() < 1000 || b.size() < 1000 || a == b) return 1;
  const char* bad[] = {"", "chem-mech 2", "chem-mech 1\nELEMENTS 1\nH 1.008\nSPECIES 1\nA 9 9 9",
                       "chem-mech 1\nELEMENTS 0\n"};
  for (const char* t : bad) {
    chemgpu::HostMech h2;
    if (parse_mechanism(t, h2) == CHEM_OK) {
      std::cerr << "malformed text accepted\n";
      return 1;
    }
  }
  std::cout << "host loader sanitizer run ok: " << a.size() << " bytes of generated source\n";
  return 0;
}
