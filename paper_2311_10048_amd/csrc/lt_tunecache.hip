// Tile choices of the contraction autotuners, persisted across processes.
//
// When the environment variable LTRIPLES_TUNE_CACHE names a file, the first
// lookup reads it and every new choice rewrites it (to a temporary file, then
// renamed over the old one).  The file is JSON with one entry per line:
//   {"ltriples_tune_cache": 1, "entries": [
//    {"arch": "gfx950:sramecc+:xnack-", "family": "bf16", "key": [3, 0, 10, 16], "cfg": 6},
//    ...
//   ]}
// An entry applies to every device of that architecture name.  Lines that do
// not parse as an entry are ignored, so a damaged file only loses choices.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <unistd.h>

#include "lt_internal.h"

namespace lt {
namespace {

struct Entry {
  std::string arch, family;
  int key[4];
  int cfg;
};

std::mutex g_mu;
bool g_loaded = false;
std::string g_path;
std::vector<Entry> g_entries;
std::map<int, std::string> g_arch;   // device index -> architecture name

const char* arch_of(int dev) {
  auto it = g_arch.find(dev);
  if (it != g_arch.end()) return it->second.c_str();
  hipDeviceProp_t p;
  std::string a = "unknown";
  if (hipGetDeviceProperties(&p, dev) == hipSuccess) a = p.gcnArchName;
  return (g_arch[dev] = a).c_str();
}

void load_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* p = getenv("LTRIPLES_TUNE_CACHE");
  if (!p || !*p) return;
  g_path = p;
  FILE* f = fopen(p, "r");
  if (!f) return;
  char line[512];
  while (fgets(line, sizeof(line), f)) {
    char arch[128], fam[32];
    Entry e;
    if (sscanf(line, " {\"arch\": \"%127[^\"]\", \"family\": \"%31[^\"]\", \"key\": [%d, %d, %d, %d], \"cfg\": %d}",
               arch, fam, &e.key[0], &e.key[1], &e.key[2], &e.key[3], &e.cfg) == 7 && e.cfg >= 0) {
      e.arch = arch;
      e.family = fam;
      g_entries.push_back(e);
    }
  }
  fclose(f);
}

Entry* find_locked(const char* arch, const char* family, const int* k) {
  for (auto& e : g_entries)
    if (e.arch == arch && e.family == family && !memcmp(e.key, k, sizeof(e.key))) return &e;
  return nullptr;
}

void save_locked() {
  if (g_path.empty()) return;
  const std::string tmp = g_path + ".tmp." + std::to_string((long)getpid());
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return;
  fprintf(f, "{\"ltriples_tune_cache\": 1, \"entries\": [\n");
  for (size_t n = 0; n < g_entries.size(); ++n) {
    const Entry& e = g_entries[n];
    fprintf(f, " {\"arch\": \"%s\", \"family\": \"%s\", \"key\": [%d, %d, %d, %d], \"cfg\": %d}%s\n", e.arch.c_str(),
            e.family.c_str(), e.key[0], e.key[1], e.key[2], e.key[3], e.cfg, n + 1 < g_entries.size() ? "," : "");
  }
  fprintf(f, "]}\n");
  const bool ok = fclose(f) == 0;
  if (ok) (void)rename(tmp.c_str(), g_path.c_str());
  else (void)remove(tmp.c_str());
}

}  // namespace

int tune_cache_get(const char* family, int dev, int k0, int k1, int k2, int k3) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  if (g_path.empty()) return -1;
  const int k[4] = {k0, k1, k2, k3};
  const Entry* e = find_locked(arch_of(dev), family, k);
  return e ? e->cfg : -1;
}

void tune_cache_put(const char* family, int dev, int k0, int k1, int k2, int k3, int cfg) {
  std::lock_guard<std::mutex> lk(g_mu);
  load_locked();
  if (g_path.empty()) return;
  const int k[4] = {k0, k1, k2, k3};
  const char* arch = arch_of(dev);
  if (Entry* e = find_locked(arch, family, k)) e->cfg = cfg;
  else g_entries.push_back({arch, family, {k0, k1, k2, k3}, cfg});
  save_locked();
}

}  // namespace lt
