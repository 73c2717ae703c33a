// Registry of the compiled Stockham specialisations (all parts, both dtypes).
#include "internal.h"

namespace fftc {

#define DECL(dt, p) const SpecEntry* spec_part_##dt##_##p(int* count);
DECL(c64, 0) DECL(c64, 1) DECL(c64, 2) DECL(c64, 3)
DECL(c128, 0) DECL(c128, 1) DECL(c128, 2) DECL(c128, 3)
#undef DECL

const SpecEntry* spec_part(int dtype, int part, int* count) {
    using Fn = const SpecEntry* (*)(int*);
    static const Fn c64[kSpecParts] = {spec_part_c64_0, spec_part_c64_1, spec_part_c64_2, spec_part_c64_3};
    static const Fn c128[kSpecParts] = {spec_part_c128_0, spec_part_c128_1, spec_part_c128_2, spec_part_c128_3};
    *count = 0;
    if (part < 0 || part >= kSpecParts) return nullptr;
    return dtype == FFTC_C128 ? c128[part](count) : c64[part](count);
}

const SpecEntry* serve_table_c64(int* count);
const SpecEntry* serve_table_c128(int* count);

const SpecEntry* find_serve(int dtype, int64_t n, const std::vector<int>& rs) {
    for (int w = 0; w < 2; ++w) {  // the powers of two's preferred lists, then the wide lists
        int cnt = 0;
        const SpecEntry* tab = w ? wide_serve_table(dtype, &cnt)
                                 : (dtype == FFTC_C128 ? serve_table_c128(&cnt) : serve_table_c64(&cnt));
        for (int i = 0; i < cnt; ++i) {
            const SpecEntry& e = tab[i];
            if (e.n != n || e.nr != (int)rs.size()) continue;
            bool same = true;
            for (int q = 0; q < e.nr; ++q) same = same && e.radices[q] == rs[q];
            if (same) return &e;
        }
    }
    return nullptr;
}

const SpecEntry* layout_table_c64(int* count);
const SpecEntry* layout_table_c128(int* count);

const SpecEntry* find_layout(int dtype, int64_t n, const std::vector<int>& rs) {
    int cnt = 0;
    const SpecEntry* tab = dtype == FFTC_C128 ? layout_table_c128(&cnt) : layout_table_c64(&cnt);
    for (int i = 0; i < cnt; ++i) {
        const SpecEntry& e = tab[i];
        if (e.n != n || e.nr != (int)rs.size()) continue;
        bool same = true;
        for (int q = 0; q < e.nr; ++q) same = same && e.radices[q] == rs[q];
        if (same) return &e;
    }
    return nullptr;
}

const FourStepEntry* fourstep_table_c64(int* count);
const FourStepEntry* fourstep_table_c128(int* count);
const FourStepEntry* colpass_table_c64(int* count);
const FourStepEntry* colpass_table_c128(int* count);

const FourStepEntry* find_colpass(int dtype, int64_t len, const std::vector<int>& rs) {
    int cnt = 0;
    const FourStepEntry* tab = dtype == FFTC_C128 ? colpass_table_c128(&cnt) : colpass_table_c64(&cnt);
    for (int i = 0; i < cnt; ++i) {
        const FourStepEntry& e = tab[i];
        if (e.len != len || e.nr != (int)rs.size()) continue;
        bool same = true;
        for (int q = 0; q < e.nr; ++q) same = same && e.radices[q] == rs[q];
        if (same) return &e;
    }
    return nullptr;
}

const OrderEntry* order_table_c64(int* count);
const OrderEntry* order_table_c128(int* count);

const OrderEntry* order_table(int dtype, int* count) {
    return dtype == FFTC_C128 ? order_table_c128(count) : order_table_c64(count);
}

const OrderEntry* find_order(int dtype, int64_t n, int order, int radix) {
    int cnt = 0;
    const OrderEntry* tab = order_table(dtype, &cnt);
    for (int i = 0; i < cnt; ++i)
        if (tab[i].n == n && tab[i].order == order && tab[i].radix == radix) return &tab[i];
    return nullptr;
}

const FourStepEntry* find_fourstep(int dtype, int64_t len, const std::vector<int>& rs) {
    int cnt = 0;
    const FourStepEntry* tab = dtype == FFTC_C128 ? fourstep_table_c128(&cnt) : fourstep_table_c64(&cnt);
    for (int i = 0; i < cnt; ++i) {
        const FourStepEntry& e = tab[i];
        if (e.len != len || e.nr != (int)rs.size()) continue;
        bool same = true;
        for (int q = 0; q < e.nr; ++q) same = same && e.radices[q] == rs[q];
        if (same) return &e;
    }
    return nullptr;
}

}  // namespace fftc
