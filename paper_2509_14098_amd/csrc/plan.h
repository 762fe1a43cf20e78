// Plan tables: what the host planner hands to the GPU kernels.
//
// A plan is the paper's partition tree flattened (Section 4.3, Fig. 6):
//   level 1  partitions  — a set T of tile qubits that stays on chip for one
//                          sweep over the state (the LDS level); the other
//                          n - |T| qubits index the tiles;
//   level 2  stages      — inside a partition, a set of at most R qubits held
//                          in each thread's registers (the register level);
//                          the rest of T is spread over lanes and waves;
//   ops                  — the partition's gates, lowered to the location of
//                          their qubits in the stage's layout.
// Both levels come from the same closeness-centrality greedy partitioner
// applied recursively (Section 4.2: the algorithm is re-invoked on each
// partition for the next memory level).
#pragma once
#include <cstdint>

namespace qsv {

// Register-level op kinds.  The gate class decides the kernel path.
enum OpKind : uint8_t {
    OP_U1 = 1,   // dense complex 2x2 on a register qubit
    OP_R1 = 2,   // real 2x2 on a register qubit
    OP_D1 = 3,   // diagonal 2x2 on a qubit anywhere
    OP_CX = 4,   // X on a register target when the control (anywhere) is 1
    OP_CU = 5,   // general 2x2 on a register target when the control is 1
    OP_CZ = 6,   // -1 when both qubits (anywhere) are 1
    OP_D2 = 7,   // diagonal 4x4 on two qubits anywhere
    OP_U2 = 8,   // dense 4x4 on two register qubits
    OP_SWAP = 9, // exchange of two register qubits
    OP_DREG = 10, // diagonal over the register index: 2^R complex entries, same for every thread
    OP_LAYER = 11, // register diagonal, then rotations on the register slots in mask a
    OP_CZ_RT = 12, // CZ between register slot a and thread or tile-index qubit b
    OP_CZ_TT = 13, // CZ between two thread or tile-index qubits
    OP_CX_T = 14,  // CX with a thread or tile-index control a, target register slot b
    OP_D1_T = 15,  // diagonal 2x2 on a thread or tile-index qubit
    OP_D2_RT = 16, // diagonal 4x4 on register slot a and thread or tile-index qubit b
    OP_D2_TT = 17, // diagonal 4x4 on two thread or tile-index qubits
};

// Location of a qubit in a stage layout: register slot, thread-id bit, or a
// bit of the tile index (outside the tile).
constexpr int32_t LOC_REG = 0x00, LOC_THR = 0x40, LOC_GLB = 0x80, LOC_MASK = 0xC0;

// Generator of a parameterised rotation exp(-i a P / 2), for the adjoint.
enum GenKind : uint8_t { GEN_NONE = 0, GEN_X = 1, GEN_Y = 2, GEN_Z = 3, GEN_ZZ = 4 };

// Every field of the device tables is 32 bits wide: byte fields let the
// compiler address neighbouring words from an unaligned scalar base, which the
// scalar memory unit does not honour (observed on gfx950 as wrong matrix
// offsets).
struct DevOp {            // 32 bytes
    int32_t kind;         // OpKind
    int32_t a;            // first location: target of U1/R1/D1, control of CX/CU, q0 of D2/CZ/U2/SWAP
    int32_t b;            // second location: target of CX/CU, q1 of D2/CZ/U2/SWAP
    int32_t gen;          // GenKind of a parameterised rotation, else GEN_NONE
    int32_t mat;          // float offset of the gate matrix in the matrix pool
    int32_t grad_slot;    // slot of this gate's gradient partial, -1 if none
    int32_t gate;         // gate index in the circuit
    int32_t flags;        // OP_D2_RT: 1 if the entries with slot bit 0 are exactly 1 (only bit-1 amplitudes change)
};

constexpr int MAX_R = 5;       // register qubits per thread (2^5 amplitudes)
constexpr int MAX_LW = 10;     // log2 threads per workgroup
constexpr int MAX_T = 15;      // tile qubits

struct DevStage {         // 104 bytes
    int32_t op_begin, op_end;
    int32_t regpos[8];    // canonical tile position of register slot j
    int32_t thrpos[16];   // canonical tile position of thread-id bit b
};

// Per-partition launch descriptor, passed by value to the sweep kernels.
struct DevPart {
    int32_t stage_begin, stage_end;
    int32_t t;            // tile qubits
    int32_t n_glb;        // n - t tile-index bits
    int32_t tq[16];       // qubit at canonical tile position c, c < t
    int32_t gq[48];       // qubit at tile-index bit b, b < n - t
};

// Pauli sums grouped by X mask, in the form the reduction kernels read.
struct DevTerm {
    double cre, cim;      // coeff * i^{#Y}
    uint64_t z_mask;
    uint32_t zt;          // expectation passes: the Z/Y mask on the pass's tile positions
    int32_t slot;         // expectation passes, diagonal groups: zt's bits at tile positions 0, 10, 11 (3 bits)
};
struct DevGroup {
    uint64_t x_mask;
    int32_t term_begin, term_end;
    int32_t xt;           // expectation passes: X mask in tile positions, -1 for partners read from HBM
    int32_t pad;
};
// One pass of qsv_expect over the state: tile qubits and the groups it handles.
struct DevPass {
    uint64_t tile_mask;
    int32_t g_begin, g_end;
    int32_t has_x;        // a group needs partner amplitudes from the LDS tile
    int32_t staged;       // its groups and terms fit EXPECT_LDS_GROUPS / EXPECT_LDS_TERMS (read from LDS copies)
};

// Matrix pool layout: a 2x2 gate takes 8 floats (row-major re,im), a 4x4
// gate 32 floats (local index j = b(q0) + 2 b(q1)), a register diagonal 2^R
// complex entries; every entry starts at a multiple of 8 floats.  OP_LAYER:
// 2^R complex diagonal entries, then the shear parameters (t, s) of the
// rotation on every register slot j at 2 j (zero where slot j has none; the
// op's field a holds the mask of slots with a rotation).

}  // namespace qsv
