"""The free list behind the tail kernel's per-plan exchange regions
(csrc/region_list.h, host-only code): two plans alive at once hold disjoint
regions, a destroyed plan's region is reused, never freed.  Compiled with g++
and run on the CPU."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

PROG = r'''
#include "region_list.h"
#include <cstdio>
#include <cstdlib>
#include <vector>
using l1::RegionList;
static std::vector<void*> made;
static void* alloc(size_t n) { void* p = std::malloc(n); made.push_back(p); return p; }
static bool disjoint(char* a, size_t na, char* b, size_t nb) { return a + na <= b || b + nb <= a; }
int main() {
  RegionList L;
  size_t ga = 0, gb = 0, gc = 0, gd = 0;
  char* a = (char*)L.get(1000, alloc, &ga);   // plan A
  char* b = (char*)L.get(1000, alloc, &gb);   // plan B, alive at the same time
  if (!a || !b || a == b || ga < 1000 || gb < 1000 || !disjoint(a, ga, b, gb)) return 1;
  L.put(a, ga);                               // plan A destroyed
  char* c = (char*)L.get(500, alloc, &gc);    // plan C reuses A's region
  if (c != a || gc != ga || made.size() != 2) return 2;
  char* d = (char*)L.get(4000, alloc, &gd);   // too large for any free region: a new one
  if (d == a || d == b || made.size() != 3 || !disjoint(d, gd, b, gb) || !disjoint(d, gd, c, gc)) return 3;
  L.put(b, gb); L.put(d, gd);
  size_t ge = 0;
  char* e = (char*)L.get(900, alloc, &ge);    // the smallest free region that fits
  if (e != b || L.free_count() != 1) return 4;
  std::puts("ok");
  return 0;
}
'''


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_regions_are_disjoint_and_reused():
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "t.cpp")
        open(src, "w").write(PROG)
        exe = os.path.join(d, "t")
        subprocess.run(["g++", "-std=c++17", "-O1", "-I", os.path.join(ROOT, "paper_1007_3753_amd", "csrc"),
                        src, "-o", exe, "-pthread"], check=True)
        r = subprocess.run([exe], capture_output=True, text=True)
        assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stdout)
