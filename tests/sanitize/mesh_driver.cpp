// Host-only driver of the mesh setup (macro-primitive graph, level layouts,
// ghost table, coarse tables), built with AddressSanitizer and
// UndefinedBehaviorSanitizer by tests/test_sanitize_host.py.
//
// Input (stdin, whitespace separated): nv nf max_level coarse_level, then nv
// coordinate pairs, then nf vertex triples.  Output: "ERR <message>" if the
// setup rejects the mesh, else "OK" followed by one line per level:
// level n_all n_int total n_ghost_copies.
#include <cstdio>
#include <iostream>
#include <vector>

#include "hhg_mesh.hpp"

int main() {
    int nv = 0, nf = 0, L = 0, lc = 0;
    if (!(std::cin >> nv >> nf >> L >> lc)) return 2;
    std::vector<double> vxy(2 * (size_t)(nv > 0 ? nv : 0));
    std::vector<int32_t> tri(3 * (size_t)(nf > 0 ? nf : 0));
    for (auto& v : vxy) std::cin >> v;
    for (auto& t : tri) std::cin >> t;
    hhg::MeshData m;
    const std::string err = m.build(vxy.data(), nv, tri.data(), nf, L, lc);
    if (!err.empty()) {
        std::printf("ERR %s\n", err.c_str());
        return 0;
    }
    std::printf("OK\n");
    for (int l = 1; l <= m.L; ++l) {
        const hhg::LevelHost& H = m.lv[l];
        std::printf("%d %lld %lld %lld %lld\n", l, (long long)H.n_all, (long long)H.n_int,
                    (long long)H.total, (long long)H.gdst.size());
    }
    return 0;
}
