// Formula plans: the paper's Kronecker-product notation (Section IV-A: the
// DSL of Listing 1 with the grammar of Listing 2) parsed, shape-checked
// (Kronecker sizes multiply, a matrix product needs equal sizes), folded back
// to DFT_n wherever a sub-formula is the Eq. 2 factorisation of one, and
// lowered to passes I_p (x) E (x) I_q with E elementary.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "internal.h"

namespace fftc {

enum FormulaPassKind {
    FP_DFT = 0,     // E = DFT_r, r a codelet radix: in place, one group per thread
    FP_STAGE = 1,   // one Stockham stage (radix r after ns) of DFT_n: out of place
    FP_DIRECT = 2,  // E = DFT_n summed directly, w_n^t from a table: out of place
    FP_DIAG = 3,    // E = D^n_a: element i a + j times w_n^{i j} (table): in place
    FP_PERM = 4,    // E = Pi^n_a: (Pi x)[i (n/a) + j] = x[j a + i]: out of place
    FP_COPY = 5     // identity (a formula with no other pass): out of place
};

struct FormulaPass {
    int kind = FP_COPY;
    int64_t n = 1;      // size of E
    int r = 0;          // DFT / STAGE: radix
    int64_t ns = 0;     // STAGE: product of the earlier radices
    int64_t a = 0;      // DIAG: M of D^n_M;  PERM: K of Pi^n_K
    int64_t p = 1, q = 1;  // I_p (x) E (x) I_q within one vector
    int64_t twoff = -1;    // first table entry (-1: no table)
};

struct FormulaProgram {
    int64_t dim = 0;                  // length of the vectors the formula acts on
    // The whole formula equals I_fold_p (x) DFT_fold_n (after folding): it
    // runs as fold_p batched transforms of the ordinary plan.
    bool folded = false;
    int64_t fold_n = 0, fold_p = 0;
    std::vector<FormulaPass> passes;  // in application order (rightmost factor first)
    std::vector<TwSegment> tables;
    int64_t table_entries = 0;
    std::string canonical;            // the formula after folding, for describe
};

// Parse, check and lower.  flags: FFTC_FORMULA_* of fftc.h.  Host only.
fftc_status compile_formula(const std::string& text, int flags, int dtype, FormulaProgram* prog);
std::string describe_formula(const FormulaProgram& prog);

// ---- execution (formula.hip) ----------------------------------------------
struct FormulaExec;  // device pass list, table and launch shape
// kernels: launches per execution (1: the whole formula in one LDS kernel).
fftc_status formula_prepare(const FormulaProgram& prog, int dtype, int64_t batch, int flags,
                            FormulaExec** out, size_t* table_bytes, size_t* scratch_bytes, int* kernels);
fftc_status formula_launch(FormulaExec* fx, const void* in, void* out, int64_t batch, bool inverse,
                           hipStream_t s);
void formula_destroy(FormulaExec* fx);
// Largest vector the one-kernel (LDS-resident) path takes for dtype.
int64_t formula_lds_max_dim(int dtype);

}  // namespace fftc
