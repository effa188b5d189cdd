// Tuning cache: launch geometries chosen by the autotuner, persisted as JSON.
#pragma once
#include <string>

#include "../../include/rdct.h"

namespace rdct {

// File: $RDCT_TUNING_CACHE, else $HOME/.cache/rdct_tuning.json.
std::string tune_cache_path();
bool tune_cache_lookup(const std::string& key, rdct_tuning_t* out);
void tune_cache_store(const std::string& key, const rdct_tuning_t& t, float us);

}  // namespace rdct
