* Maximisation with an objective constant, RANGES on every row type and
* sign, integrality markers and integer bounds (read as the relaxation).
NAME RANGEMAX
OBJSENSE
    MAX
ROWS
 N  PROFIT
 G  R1
 L  R2
 E  R3
 E  R4
COLUMNS
    X1  PROFIT  3.0   R1  1.0
    X1  R2      1.0
    X2  PROFIT  2.0   R1  1.0
    X2  R3      1.0
    MARKER  'MARKER'  'INTORG'
    X3  PROFIT  -1.0  R2  2.0
    X3  R4      1.0
    MARKER  'MARKER'  'INTEND'
    X4  PROFIT  1.0   R3  1.0
    X4  R4      -1.0
RHS
    RHS  PROFIT  -10.0
    RHS  R1  1.0  R2  8.0
    RHS  R3  2.0  R4  0.5
RANGES
    RNG  R1  5.0
    RNG  R2  -3.0
    RNG  R3  4.0
    RNG  R4  -2.0
BOUNDS
 UP BND X1 4.0
 MI BND X2
 UP BND X2 3.0
 LI BND X3 1
 UI BND X3 5
 FR BND X4
ENDATA
