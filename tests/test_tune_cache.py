"""Host logic of the tuning cache (rdct_tune.cpp), built with g++ into a small
driver: stores and lookups round-trip, a stored key is overwritten, entries
written before the layout field existed read as the strided layout, lines the
scanner does not understand are skipped, and a missing file finds nothing."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1402_6034_amd", "csrc")

DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "rdct_tune.h"

// store KEY WPG WPC LAYOUT US | lookup KEY
int main(int argc, char** argv) {
  if (argc >= 7 && !strcmp(argv[1], "store")) {
    rdct_tuning_t t{};
    t.waves_per_wg = atoi(argv[3]);
    t.wgs_per_cu = atoi(argv[4]);
    t.layout = atoi(argv[5]);
    rdct::tune_cache_store(argv[2], t, (float)atof(argv[6]));
    return 0;
  }
  if (argc >= 3 && !strcmp(argv[1], "lookup")) {
    rdct_tuning_t t{};
    t.use_graph = 7;
    if (!rdct::tune_cache_lookup(argv[2], &t)) {
      printf("missing\n");
      return 0;
    }
    printf("%d %d %d %d\n", t.waves_per_wg, t.wgs_per_cu, t.layout, t.use_graph);
    return 0;
  }
  return 2;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("tune")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    subprocess.run([gxx, "-std=c++17", "-O1", "-I", CSRC, str(src),
                    os.path.join(CSRC, "rdct_tune.cpp"), "-o", str(exe), "-lpthread"],
                   check=True, capture_output=True)
    return str(exe)


def run(driver, cache, *args):
    env = dict(os.environ, RDCT_TUNING_CACHE=str(cache))
    out = subprocess.run([driver, *map(str, args)], env=env, check=True, capture_output=True,
                         text=True)
    return out.stdout.strip()


def test_store_lookup_and_overwrite(driver, tmp_path):
    cache = tmp_path / "sub" / "dir" / "tune.json"      # parent folders are created
    assert run(driver, cache, "lookup", "gfx950/a") == "missing"
    run(driver, cache, "store", "gfx950/a", 1, 4, 1, 1312.5)
    run(driver, cache, "store", "gfx950/b", 4, 1, 2, 65.4)
    # Lookups never turn graph replay on: plain launches are the default.
    assert run(driver, cache, "lookup", "gfx950/a") == "1 4 1 0"
    assert run(driver, cache, "lookup", "gfx950/b") == "4 1 2 0"
    run(driver, cache, "store", "gfx950/a", 2, 8, 2, 1200.0)
    assert run(driver, cache, "lookup", "gfx950/a") == "2 8 2 0"
    assert run(driver, cache, "lookup", "gfx950/b") == "4 1 2 0"
    text = cache.read_text()
    assert text.count('"key"') == 2 and '"layout": 2' in text
    assert not os.path.exists(str(cache) + ".tmp")


def test_old_entries_and_unknown_lines(driver, tmp_path):
    cache = tmp_path / "tune.json"
    cache.write_text(
        '{"rdct_tuning": 1, "entries": [\n'
        '  {"key": "gfx950/old", "waves_per_wg": 2, "wgs_per_cu": 4, "us": 80.0},\n'
        '  {"key": "gfx950/broken", "waves_per_wg": 2},\n'
        '  not json at all\n'
        '  {"key": "gfx950/new", "waves_per_wg": 4, "wgs_per_cu": 1, "layout": 2, "us": 65.0}\n'
        ']}\n')
    assert run(driver, cache, "lookup", "gfx950/old") == "2 4 1 0"     # strided
    assert run(driver, cache, "lookup", "gfx950/broken") == "missing"
    assert run(driver, cache, "lookup", "gfx950/new") == "4 1 2 0"
    # A store rewrites the file in the current format and keeps the readable entries.
    run(driver, cache, "store", "gfx950/x", 1, 2, 1, 10.0)
    text = cache.read_text()
    assert "broken" not in text and "not json" not in text
    assert run(driver, cache, "lookup", "gfx950/old") == "2 4 1 0"
    assert '"key": "gfx950/old", "waves_per_wg": 2, "wgs_per_cu": 4, "layout": 1' in text
