"""OpenQASM 2 subset front end: text -> gate array for qsv_partition.

The paper's tool takes circuits as OpenQASM (Section 4.1: quantum registers,
then one gate per line).  This reader accepts the subset that maps onto the
gate kinds of the C interface:

  OPENQASM 2.0;  include "...";  qreg name[size];  creg name[size];
  one- and two-qubit gates from the standard library, one per statement:
    id x y z h s sdg t tdg sx rx(a) ry(a) rz(a) p(a) u1(a) u3(a,b,c) u(a,b,c)
    cx CX cy cz cp(a) cu1(a) swap rzz(a)
  barrier is skipped; measure is skipped when no later gate acts on the
  measured qubit (the library computes the amplitudes before measurement; it
  does not sample); reset and gates after a measurement are rejected.

Reading of `rz`: qelib1.inc defines rz(a) as u1(a) = diag(1, e^{ia}); this
reader takes it as the rotation RZ(a) = exp(-i a Z / 2) = diag(e^{-ia/2},
e^{ia/2}) instead (the convention of Qiskit, through which the paper parses
its circuits, Section 4.1).  The two differ by the global phase e^{-ia/2}:
every expectation value and probability is the same, amplitudes are not.
`u1` and `p` are the phase gate diag(1, e^{ia}) as in qelib1.

Qubits of successive qreg declarations are numbered consecutively: qubit q of
the circuit is bit q of the amplitude index.  Angle expressions may use
numbers, pi, + - * / and parentheses; they are evaluated with a small
arithmetic interpreter (no Python eval).  Gate definitions (`gate ... { }`),
classical conditions and multi-register broadcasting are rejected with a
ValueError naming the line.
"""
from __future__ import annotations

import ast
import math
import operator
import re

import numpy as np

from .binding import GATE_DTYPE, KIND

_ONE = {"x": "X", "y": "Y", "z": "Z", "h": "H", "s": "S", "sdg": "SDG", "t": "T", "tdg": "TDG", "sx": "SX"}
_ONE_PARAM = {"rx": "RX", "ry": "RY", "rz": "RZ", "p": "P", "u1": "P"}
_TWO = {"cx": "CX", "CX": "CX", "cy": "CY", "cz": "CZ", "swap": "SWAP"}
_TWO_PARAM = {"cp": "CP", "cu1": "CP", "rzz": "RZZ"}
_SKIP = ("barrier", "creg", "include", "OPENQASM")

_BINOPS = {ast.Add: operator.add, ast.Sub: operator.sub, ast.Mult: operator.mul, ast.Div: operator.truediv,
           ast.Pow: operator.pow}


def _angle(text: str) -> float:
    """Value of an angle expression made of numbers, pi and + - * / ** ( )."""
    def ev(node):
        if isinstance(node, ast.Expression):
            return ev(node.body)
        if isinstance(node, ast.Constant) and isinstance(node.value, (int, float)):
            return float(node.value)
        if isinstance(node, ast.Name) and node.id == "pi":
            return math.pi
        if isinstance(node, ast.UnaryOp) and isinstance(node.op, (ast.USub, ast.UAdd)):
            v = ev(node.operand)
            return -v if isinstance(node.op, ast.USub) else v
        if isinstance(node, ast.BinOp) and type(node.op) in _BINOPS:
            return _BINOPS[type(node.op)](ev(node.left), ev(node.right))
        raise ValueError(f"unsupported angle expression: {text!r}")
    return ev(ast.parse(text.strip(), mode="eval"))


def parse(text: str):
    """Returns (n_qubits, gates) with gates in the qsv_gate layout."""
    regs, n = {}, 0
    rows = []
    measured = set()
    # statements end with ';' (comments removed first)
    body = re.sub(r"//[^\n]*", "", text)
    for lineno, stmt in enumerate(s.strip() for s in body.split(";")):
        if not stmt:
            continue
        if stmt.startswith(_SKIP):
            continue
        if stmt.startswith("reset"):
            raise ValueError(f"statement {lineno + 1}: reset is not unitary")
        mm = re.fullmatch(r"measure\s+(\w+)\s*\[\s*(\d+)\s*\]\s*->\s*\w+\s*\[\s*\d+\s*\]", stmt)
        if mm:
            if mm.group(1) not in regs:
                raise ValueError(f"statement {lineno + 1}: unknown register in {stmt!r}")
            measured.add(regs[mm.group(1)][0] + int(mm.group(2)))
            continue
        if stmt.startswith(("gate ", "opaque ", "if")) or "{" in stmt:
            raise ValueError(f"statement {lineno + 1}: gate definitions and conditions are not supported: {stmt!r}")
        m = re.fullmatch(r"qreg\s+(\w+)\s*\[\s*(\d+)\s*\]", stmt)
        if m:
            regs[m.group(1)] = (n, int(m.group(2)))
            n += int(m.group(2))
            continue
        m = re.fullmatch(r"(\w+)\s*(?:\((.*)\))?\s+(.+)", stmt, re.S)
        if not m:
            raise ValueError(f"statement {lineno + 1}: cannot parse {stmt!r}")
        name, args, operands = m.group(1), m.group(2), m.group(3)
        angles = [_angle(a) for a in args.split(",")] if args else []
        qubits = []
        for op in operands.split(","):
            mq = re.fullmatch(r"\s*(\w+)\s*\[\s*(\d+)\s*\]\s*", op)
            if not mq or mq.group(1) not in regs:
                raise ValueError(f"statement {lineno + 1}: bad qubit operand {op!r} (whole-register operands are "
                                 f"not supported)")
            base, size = regs[mq.group(1)]
            if int(mq.group(2)) >= size:
                raise ValueError(f"statement {lineno + 1}: {op.strip()} is out of range")
            qubits.append(base + int(mq.group(2)))

        if measured.intersection(qubits):
            raise ValueError(f"statement {lineno + 1}: gate on a measured qubit")

        def need(nq, na):
            if len(qubits) != nq or len(angles) != na:
                raise ValueError(f"statement {lineno + 1}: {name} takes {nq} qubit(s) and {na} angle(s)")

        if name == "id":
            need(1, 0)
            continue
        if name in _ONE:
            need(1, 0)
            rows.append((_ONE[name], qubits, []))
        elif name in _ONE_PARAM:
            need(1, 1)
            rows.append((_ONE_PARAM[name], qubits, angles))
        elif name in ("u3", "u", "U"):
            need(1, 3)
            rows.append(("U3", qubits, angles))
        elif name in _TWO:
            need(2, 0)
            rows.append((_TWO[name], qubits, []))
        elif name in _TWO_PARAM:
            need(2, 1)
            rows.append((_TWO_PARAM[name], qubits, angles))
        else:
            raise ValueError(f"statement {lineno + 1}: unsupported gate {name!r}")
    gates = np.zeros(len(rows), dtype=GATE_DTYPE)
    for i, (kind, qubits, angles) in enumerate(rows):
        gates[i]["kind"] = KIND[kind]
        gates[i]["q0"] = qubits[0]
        gates[i]["q1"] = qubits[1] if len(qubits) > 1 else -1
        gates[i]["param"] = -1
        a = np.zeros(3)
        a[:len(angles)] = angles
        gates[i]["angle"] = a
    return n, gates


# gate kind -> OpenQASM name (the fixed-angle kinds parse() reads)
_QASM_NAME = {"X": "x", "Y": "y", "Z": "z", "H": "h", "S": "s", "SDG": "sdg", "T": "t", "TDG": "tdg", "SX": "sx",
              "RX": "rx", "RY": "ry", "RZ": "rz", "P": "p", "U3": "u3", "CX": "cx", "CY": "cy", "CZ": "cz",
              "SWAP": "swap", "CP": "cp", "RZZ": "rzz"}
_N_ANGLES = {"RX": 1, "RY": 1, "RZ": 1, "P": 1, "CP": 1, "RZZ": 1, "U3": 3}


def dump(n_qubits: int, gates) -> str:
    """OpenQASM 2 text of a gate array made of the kinds parse() reads (fixed angles)."""
    kind_name = {v: k for k, v in KIND.items()}
    lines = ["OPENQASM 2.0;", 'include "qelib1.inc";', f"qreg q[{n_qubits}];"]
    for g in np.asarray(gates):
        name = kind_name[int(g["kind"])]
        if name not in _QASM_NAME or int(g["param"]) >= 0:
            raise ValueError(f"gate kind {name} (or a theta parameter) has no OpenQASM form here")
        nargs = _N_ANGLES.get(name, 0)
        args = "(" + ",".join(repr(float(a)) for a in g["angle"][:nargs]) + ")" if nargs else ""
        qs = [int(g["q0"])] + ([int(g["q1"])] if int(g["q1"]) >= 0 else [])
        lines.append(f"{_QASM_NAME[name]}{args} " + ",".join(f"q[{q}]" for q in qs) + ";")
    return "\n".join(lines) + "\n"
