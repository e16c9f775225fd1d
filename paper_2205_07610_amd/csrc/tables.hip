// Persisted variant tables (the autotuner's result, section 11 of the
// batching runtime; not in the paper): the three modes' per-length-bin
// full-DP variants and the automatic setting's measured cell type per mode
// as one versioned, checksummed blob, so that a table tuned once can be
// loaded by later processes instead of tuning again.
//
// Layout (little-endian), 68 bytes:
//   char magic[8] = "ASVARTAB"; uint32 version = 2; uint32 n_modes = 3;
//   uint32 n_bins = 12; uint32 n_variants = 6; int8 table[3][12];
//   int8 half_pref[3]; uint8 zero;
//   uint32 checksum (FNV-1a 32 of bytes 0..63 with the checksum field zero).
// Version 1 (64 bytes: no half_pref, checksum at byte 60) still loads and
// clears the measured cell types.  The tables are read and written through
// as_get_variants / as_set_variants and the cell types through
// as_half_cells_preference, so a loaded blob is validated exactly like
// values set directly.
#include <string.h>

#include "internal.h"

namespace {

constexpr int64_t kTabBlob = 68;
constexpr int64_t kTabBlobV1 = 64;
constexpr int kTabModes = 3;
constexpr uint32_t kTabVersion = 2;
constexpr int kTabTableOff = 24;
constexpr int kTabPrefOff = kTabTableOff + kTabModes * asmi::kLenBins;  // 60
constexpr int kTabSumOff = kTabPrefOff + 4;                              // 64
constexpr int kTabSumOffV1 = kTabPrefOff;                                // 60

uint32_t tab_fnv1a(const uint8_t *p, int64_t n) {
  uint32_t h = 2166136261u;
  for (int64_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 16777619u;
  }
  return h;
}

void put_u32(uint8_t *p, uint32_t v) {
  for (int i = 0; i < 4; ++i) p[i] = (uint8_t)(v >> (8 * i));
}
uint32_t get_u32(const uint8_t *p) {
  uint32_t v = 0;
  for (int i = 0; i < 4; ++i) v |= (uint32_t)p[i] << (8 * i);
  return v;
}

}  // namespace

static_assert(kTabSumOff + 4 == kTabBlob && kTabSumOffV1 + 4 == kTabBlobV1, "variant table blob layout");

extern "C" int64_t as_variant_tables_blob_size(void) { return kTabBlob; }

extern "C" int as_variant_tables_save(uint8_t *blob_out, int64_t blob_size) {
  if (!blob_out) return AS_ERR_NULL;
  if (blob_size < kTabBlob) return AS_ERR_ARG;
  uint8_t b[kTabBlob];
  memset(b, 0, sizeof(b));
  memcpy(b, "ASVARTAB", 8);
  put_u32(b + 8, kTabVersion);
  put_u32(b + 12, kTabModes);
  put_u32(b + 16, asmi::kLenBins);
  put_u32(b + 20, asmi::kNumVariants);
  for (int mode = 0; mode < kTabModes; ++mode) {
    const int rc = as_get_variants(mode, (int8_t *)(b + kTabTableOff + mode * asmi::kLenBins));
    if (rc) return rc;
    b[kTabPrefOff + mode] = (uint8_t)(int8_t)as_half_cells_preference(mode, 0, 0);
  }
  put_u32(b + kTabSumOff, tab_fnv1a(b, kTabBlob));
  memcpy(blob_out, b, sizeof(b));
  return AS_OK;
}

extern "C" int as_variant_tables_load(const uint8_t *blob, int64_t blob_size) {
  if (!blob) return AS_ERR_NULL;
  if (blob_size != kTabBlob && blob_size != kTabBlobV1) return AS_ERR_ARG;
  const bool v1 = blob_size == kTabBlobV1;
  uint8_t b[kTabBlob];
  memcpy(b, blob, (size_t)blob_size);
  const int sum_off = v1 ? kTabSumOffV1 : kTabSumOff;
  if (memcmp(b, "ASVARTAB", 8) != 0 || get_u32(b + 8) != (v1 ? 1u : kTabVersion) ||
      get_u32(b + 12) != kTabModes || get_u32(b + 16) != (uint32_t)asmi::kLenBins ||
      get_u32(b + 20) != (uint32_t)asmi::kNumVariants)
    return AS_ERR_ARG;
  const uint32_t sum = get_u32(b + sum_off);
  put_u32(b + sum_off, 0);
  if (tab_fnv1a(b, blob_size) != sum) return AS_ERR_ARG;
  // every value is checked before any is set, so a bad blob changes nothing
  for (int mode = 0; mode < kTabModes; ++mode) {
    for (int k = 0; k < asmi::kLenBins; ++k) {
      const int v = (int8_t)b[kTabTableOff + mode * asmi::kLenBins + k];
      if (v < -1 || v >= asmi::kNumVariants) return AS_ERR_ARG;
    }
    if (!v1) {
      const int h = (int8_t)b[kTabPrefOff + mode];
      if (h < -1 || h > 1) return AS_ERR_ARG;
    }
  }
  if (!v1 && b[kTabPrefOff + 3] != 0) return AS_ERR_ARG;
  for (int mode = 0; mode < kTabModes; ++mode) {
    const int rc = as_set_variants(mode, (const int8_t *)(b + kTabTableOff + mode * asmi::kLenBins));
    if (rc) return rc;
    const int hp = as_half_cells_preference(mode, v1 ? -1 : (int8_t)b[kTabPrefOff + mode], 1);
    if (hp < -1) return hp;
  }
  return AS_OK;
}
