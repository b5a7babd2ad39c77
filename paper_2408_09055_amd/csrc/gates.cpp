// Gate vocabulary of libqk: arity, cost class, diagonality and FP64
// matrices.  The matrices use the OpenQASM 2 definitions (the paper defines
// none); matrix index bit j belongs to the j-th listed qubit.
#include <cmath>

#include "qk_internal.hpp"

namespace qk {

int kind_arity(uint32_t kind)
{
    if (kind >= QK_NUM_KINDS) return 0;
    return kind >= QK_CX ? 2 : 1;
}

int gate_class(uint32_t kind)
{
    switch (kind) {
    case QK_H: return 0;
    case QK_X: case QK_Y: return 1;
    case QK_CX: case QK_SWAP: return 3;
    case QK_CZ: return 4;
    case QK_CP: return 5;
    case QK_RZZ: return 6;
    default: return 2;   // remaining one-qubit gates
    }
}

bool kind_is_diagonal(uint32_t kind)
{
    switch (kind) {
    case QK_Z: case QK_S: case QK_T: case QK_RZ: case QK_P:
    case QK_CZ: case QK_CP: case QK_RZZ:
        return true;
    default:
        return false;
    }
}

static cd phase(double a) { return std::polar(1.0, a); }

static void set_diag(cd* U, int dim, const cd* d)
{
    for (int r = 0; r < dim; ++r)
        for (int c = 0; c < dim; ++c) U[r * dim + c] = (r == c) ? d[r] : cd(0.0, 0.0);
}

void gate_unitary(const qk_gate& g, cd* U)
{
    const double th = g.p[0];
    const double ch = std::cos(0.5 * th), sh = std::sin(0.5 * th);
    const cd i1(0.0, 1.0);
    const double r2 = 1.0 / std::sqrt(2.0);
    switch (g.kind) {
    case QK_H: U[0] = r2; U[1] = r2; U[2] = r2; U[3] = -r2; return;
    case QK_X: U[0] = 0.0; U[1] = 1.0; U[2] = 1.0; U[3] = 0.0; return;
    case QK_Y: U[0] = 0.0; U[1] = -i1; U[2] = i1; U[3] = 0.0; return;
    case QK_RX: U[0] = ch; U[1] = -i1 * sh; U[2] = -i1 * sh; U[3] = ch; return;
    case QK_RY: U[0] = ch; U[1] = -sh; U[2] = sh; U[3] = ch; return;
    case QK_U3: {
        const double ph = g.p[1], la = g.p[2];
        U[0] = ch;
        U[1] = -phase(la) * sh;
        U[2] = phase(ph) * sh;
        U[3] = phase(ph + la) * ch;
        return;
    }
    case QK_Z: { cd d[2] = {1.0, -1.0}; set_diag(U, 2, d); return; }
    case QK_S: { cd d[2] = {1.0, i1}; set_diag(U, 2, d); return; }
    case QK_T: { cd d[2] = {1.0, phase(M_PI / 4.0)}; set_diag(U, 2, d); return; }
    case QK_RZ: { cd d[2] = {phase(-0.5 * th), phase(0.5 * th)}; set_diag(U, 2, d); return; }
    case QK_P: { cd d[2] = {1.0, phase(th)}; set_diag(U, 2, d); return; }
    case QK_CZ: { cd d[4] = {1.0, 1.0, 1.0, -1.0}; set_diag(U, 4, d); return; }
    case QK_CP: { cd d[4] = {1.0, 1.0, 1.0, phase(th)}; set_diag(U, 4, d); return; }
    case QK_RZZ: {
        // parity of the two bits selects e^{-i t/2} (even) or e^{+i t/2} (odd)
        cd d[4] = {phase(-0.5 * th), phase(0.5 * th), phase(0.5 * th), phase(-0.5 * th)};
        set_diag(U, 4, d);
        return;
    }
    case QK_CX:
    case QK_SWAP: {
        // permutation matrices: column c maps to row sigma(c)
        int sigma[4];
        if (g.kind == QK_CX) { sigma[0] = 0; sigma[1] = 3; sigma[2] = 2; sigma[3] = 1; }
        else { sigma[0] = 0; sigma[1] = 2; sigma[2] = 1; sigma[3] = 3; }
        for (int i = 0; i < 16; ++i) U[i] = 0.0;
        for (int c = 0; c < 4; ++c) U[sigma[c] * 4 + c] = 1.0;
        return;
    }
    default: return;
    }
}

}  // namespace qk
