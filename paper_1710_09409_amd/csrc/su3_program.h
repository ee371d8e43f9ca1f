// Internal interface of the expression-program kernel unit
// (su3_kprog.hip) and the host expression compiler (su3_program.cpp) for
// the host C-ABI unit.  Not installed, not part of the ABI.
#pragma once

#include "su3_internal.h"

namespace su3i {

// ------------------------------------------------ expression programs
//
// A site-local expression compiled on the host into a register program.
// Registers hold a 3x3 complex matrix; a scalar occupies entry 0 (real
// scalars keep a zero imaginary part).  Operand k is loaded into register
// k before the first instruction; instructions read registers a, b and
// write register d; the result is register `result`.
enum ProgOp : uint8_t {
    OP_CONST = 0,  // r[d] = imm[a] (scalar)
    OP_ADD_MM, OP_SUB_MM, OP_MUL_MM,
    OP_ADD_SS, OP_SUB_SS, OP_MUL_SS,
    OP_MUL_SM,     // r[d] = r[a] (scalar) * r[b] (matrix)
    OP_MUL_MS,     // r[d] = r[a] (matrix) * r[b] (scalar)
    OP_ADD_SM,     // r[d] = r[a] I + r[b]
    OP_ADD_MS,     // r[d] = r[a] + r[b] I
    OP_SUB_SM,     // r[d] = r[a] I - r[b]
    OP_SUB_MS,     // r[d] = r[a] - r[b] I
    OP_NEG_M, OP_NEG_S,
    OP_ADJ_M,      // conjugate transpose
    OP_CONJ_M,     // elementwise conjugate
    OP_CONJ_S,
    OP_TRACE,      // matrix -> complex scalar
    OP_REAL, OP_IMAG,  // scalar -> real scalar
    OP_TRANS_M,    // transpose
    NPROGOP
};

constexpr int kProgMaxOps = 8;     // operand fields
constexpr int kProgMaxInstr = 48;
constexpr int kProgMaxImm = 8;
constexpr int kProgMaxRegs = 8;

struct ProgInstr {
    uint8_t op, d, a, b;
};

// Field kinds of program operands and results.
enum FieldKind { FK_MATRIX = 0, FK_SPINOR = 1, FK_REAL = 2, FK_COMPLEX = 3 };

struct ProgArgs {
    void *z;
    const void *op[kProgMaxOps];
    Geom g[kProgMaxOps];      // per operand (entry counts differ by kind)
    Geom gz;
    uint8_t kind[kProgMaxOps];   // FieldKind
    uint8_t prec[kProgMaxOps];   // storage precision (F64, F32, C12)
    uint8_t zkind, zprec;
    uint8_t nops, ninstr, result;
    uint8_t used;                // bit k: operand k is read
    int32_t nsites;
    double imm[kProgMaxImm][2];
    ProgInstr ins[kProgMaxInstr];
};

// Kernel forms: PF_MATRIX (matrix values anywhere; one site per lane),
// PF_SCALAR (no matrix value; complex registers), PF_REAL (every value
// real: operands, intermediates and result).
enum ProgForm { PF_MATRIX = 0, PF_SCALAR = 1, PF_REAL = 2 };

// Arithmetic precision F64 (all fields F64) or F32 (F32 / C12 fields).
// Every form takes up to 8 registers; programs with matrix values run one
// site per lane, the scalar and real forms program_sites_per_lane() sites
// per lane.  block is 64, 128 or 256;
// grid * block * sites per lane >= nsites.
int program_sites_per_lane(int arith, int form);
hipError_t launch_program(int arith, int form, int nregs, int nt,
                          int block, int grid, size_t shm, const ProgArgs &a,
                          hipStream_t stream);

// Host compiler (su3_program.cpp): parse `text` over n operands of the
// given kinds (FieldKind), type-check and allocate registers.  Fills
// ins/ninstr/imm/result/nops of `out`, the result kind and the number of
// registers used; returns false with a message in *err.
struct ProgCode {
    ProgInstr ins[kProgMaxInstr];
    int ninstr;
    double imm[kProgMaxImm][2];
    int nimm;
    int result;
    int result_kind;
    int nregs;
    int nops;
    bool su3_closed;  // only products, adjoints and transposes of matrices
    bool scalar_only; // no matrix-valued operand or intermediate
    bool real_only;   // every operand, intermediate and the result real
    unsigned used;    // bit k: operand k is read
};
bool compile_program(const char *text, int nops, const int *kinds,
                     ProgCode *out, char *err, size_t errlen);

}  // namespace su3i
