// Host-side probe of the planner, built with g++ by tests/test_host_planner.py
// (no GPU): prints the closed-form kind of patterns, or the plan compiled
// for given graph statistics.
//   plan_probe kinds <k:mask> ...
//   plan_probe plans n m avg_deg nbr_deg avg_out nbr_out max_deg max_out s_pp s_pq s_pd s_qq s_qd s_dd
//              <tri 0/1> <k:mask> ...
// Each pattern line: "<k>:<mask hex> kind=<tagg kind>" or
// "<k>:<mask hex> rc=<status> ncore=<levels> local=<0/1> tagg=<kind>".
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>

#include "../../paper_2012_04553_amd/csrc/internal.hpp"

using namespace pm;

static Pat parse(const char* s) {
    Pat p;
    p.k = s[0] - '0';
    p.em = (uint32_t)strtoul(s + 2, nullptr, 16);
    p.vi = false;
    return p;
}

int main(int argc, char** argv) {
    if (argc < 2) return 2;
    if (!strcmp(argv[1], "kinds")) {
        for (int i = 2; i < argc; ++i) printf("%s kind=%d\n", argv[i], tagg_kind(parse(argv[i])));
        return 0;
    }
    if (strcmp(argv[1], "plans") || argc < 17) return 2;
    GraphStats s;
    double* f[] = {&s.n,       &s.m,       &s.avg_deg, &s.nbr_deg, &s.avg_out, &s.nbr_out, &s.max_deg,
                   &s.max_out, &s.s_pp,    &s.s_pq,    &s.s_pd,    &s.s_qq,    &s.s_qd,    &s.s_dd};
    for (int i = 0; i < 14; ++i) *f[i] = atof(argv[2 + i]);
    const bool tri = atoi(argv[16]) != 0;
    for (int i = 17; i < argc; ++i) {
        PlanInfo pi;
        std::string err;
        const int rc = compile_plan(parse(argv[i]), s, &pi, &err, tri);
        printf("%s rc=%d ncore=%d local=%d tagg=%d\n", argv[i], rc, pi.d.ncore, pi.d.local, pi.d.tagg);
    }
    return 0;
}
