// Host-side structure of one substructuring level: integer work only
// (DOF numbering, interface classification, constraint layout, pair maps).
// Floating-point work runs in the HIP kernels.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace ambddc {

enum GlobType { GLOB_FACE = 0, GLOB_EDGE = 1, GLOB_CORNER = 2 };
enum ConsKind { CONS_UNIT = 0, CONS_AVG = 1, CONS_ADAPT = 2 };

// A level's "mesh": elements over level DOFs.  Level 1: FE elements and
// mesh nodes.  Level i+1: the level-i subdomains are the elements and the
// level-i globs that carry coarse DOFs are the nodes (Section 3).
struct LevelInput {
  int n_dof = 0, n_node = 0, n_sub = 0, n_elem = 0;
  int dof_per_node = 1;
  int n_rb = 1;                               // rigid modes per subdomain
  std::vector<int> elem_sub;
  std::vector<int64_t> elem_dof_ptr;          // CSR over elements
  std::vector<int> elem_dofs;                 // level DOF id, -1 = fixed
  std::vector<int64_t> elem_node_ptr;
  std::vector<int> elem_nodes;
  std::vector<int> node_dof_ptr, node_dofs;   // free DOFs of each node
  std::vector<int> dof_comp;                  // component or -1
  std::vector<char> sub_floating;
};

struct Glob {
  int type = GLOB_FACE;
  std::vector<int> subs;    // sorted
  std::vector<int> nodes;
  std::vector<int> dofs;    // sorted level DOF ids
};

struct Constraint {
  int glob = -1;
  int kind = CONS_UNIT;
  std::vector<int> dofs;    // support (level DOF ids, ascending)
  int pair = -1, row = -1;  // adaptive: source pair and row
};

struct Sub {
  std::vector<int> dofs;    // interior (ascending) then interface (ascending)
  int nI = 0, nG = 0;
  std::vector<int> cons;    // coarse ids of C^s rows, ascending
};

struct Pair {
  int s = -1, t = -1, glob = -1;
  std::vector<int> sh_s, sh_t;      // shared DOFs: local interface index in s / t
  std::vector<int> dr_s, dr_t;      // shared coarse DOFs: row of C^s / C^t
  std::vector<int> face_s, face_t;  // support of the adaptive rows: local interface index in s / t
  std::vector<int> face_dofs;       // level ids of that support (ascending)
  std::vector<int> pc_s, pc_t;      // pair-coarse index of each row of C^s / C^t
  int n_cp = 0;
  bool both_floating = false;
  int slot_s = -1, slot_t = -1;     // position among the pairs of s / t
};

struct LevelPlan {
  LevelInput in;
  std::vector<Glob> globs;
  std::vector<Constraint> cons;
  std::vector<Sub> subs;
  std::vector<Pair> pairs;
  std::vector<int> dof_node;
  std::vector<int> sub_npairs;      // pairs per subdomain
  int n_cons_initial = 0;
};

// Initial constraint sets (Section 7 and Section 8.2's variants).
enum InitCons { INIT_CE = 0, INIT_CEF = 1, INIT_C = 2 };

// Build globs, subdomain DOF sets, initial constraints (corners; edge
// averages per component unless `init` is INIT_C; face averages for
// INIT_CEF) and pair maps.  The support of a pair's adaptive rows
// (face_dofs, face_s, face_t) is its face, or with keep_edges all DOFs the
// two subdomains share.  Returns an empty string on success, else an error
// message.
std::string build_level_plan(LevelPlan& L, int init, bool keep_edges);

// Append adaptive constraints (k[p] rows on the face of pair p) and rebuild
// the per-subdomain constraint lists and pair-coarse maps.
void add_adaptive_constraints(LevelPlan& L, const std::vector<int>& k);

// Level-(i+1) input from an enriched level-i plan and the parent map.
std::string next_level_input(const LevelPlan& L, const std::vector<int>& parent, LevelInput& out);

// Level-1 input from the mesh.
std::string level1_input(int n_nodes, int n_elems, int dof, const int32_t* elem_nodes,
                         const uint8_t* dirichlet, const int32_t* elem_to_sub, LevelInput& out,
                         std::vector<int>& free_of_full);

}  // namespace ambddc
